"""Pins of the oracle's refinement / de-refinement (Sec. 2.2): the criterion
against brute force on a grid, the closure against grading and minimality,
the state transfer against exact copies and conservation, and the whole
procedure against the static sphere trees built by the input module's own
(independent) graded construction."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I
from test_oracle_scheme import from_grid, leaf_totals, random_state, to_grid


def _cells(T):
    """{(l, x, y, z): cell index} over every cell of tree T."""
    pos = {}
    for o in range(T.n):
        i, j, k, l = (int(v) for v in T.ijkl[o])
        for c in range(8):
            pos[(l, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1))] = 8 * o + c
    return pos


def _octs(T):
    return {tuple(int(v) for v in r): o for o, r in enumerate(T.ijkl)}


@pytest.mark.parametrize("bc", [I.PERIODIC, I.OUTFLOW])
@pytest.mark.parametrize("rho_t,grad_t", [(1.4, 0.0), (0.0, 0.12), (1.6, 0.2)])
def test_criterion_brute_force_single_level(bc, rho_t, grad_t):
    """One level (no closure below it): the flags are the criterion, written
    out on the dense grid with numpy."""
    ijkl = I.uniform_tree(4)
    T = O.Tree(ijkl, bc)
    u = T.permute_cells(random_state(ijkl, 4, 41, 5.0 / 3.0))
    flags, _, _ = T.refine(u, rho_t, grad_t, 5)
    rho = to_grid(T, u)[..., 0]
    want = np.zeros(rho.shape, bool)
    if rho_t > 0:
        want |= rho > rho_t
    if grad_t > 0:
        for ax in range(3):
            for sh in (1, -1):
                if bc == I.PERIODIC:
                    n = np.roll(rho, sh, axis=ax)
                else:
                    n = np.roll(rho, sh, axis=ax)
                    edge = [slice(None)] * 3
                    edge[ax] = 0 if sh == 1 else -1
                    n[tuple(edge)] = rho[tuple(edge)]
                want |= np.abs(n - rho) / (n + rho) > grad_t
    got = np.zeros(rho.shape + (5,))
    bits = ((flags[:, None] >> np.arange(8)[None, :]) & 1).reshape(-1).astype(float)
    g = to_grid(T, np.repeat(bits[:, None], 5, axis=1))[..., 0] > 0
    assert want.any() and not want.all()
    assert np.array_equal(g, want)
    assert np.array_equal(T.last_crit, flags)


def _amr_case(seed):
    ijkl = I.sphere_tree(3, 6, (0.45, 0.5, 0.55), 0.2, I.PERIODIC)
    T = O.Tree(ijkl, I.PERIODIC)
    u = T.permute_cells(random_state(ijkl, 3, seed, 5.0 / 3.0))
    T.run(u, 5.0 / 3.0, 0.8, 2)
    return T, u


@pytest.mark.parametrize("params", [(1.3, 0.0, 7), (0.0, 0.1, 6), (1.5, 0.15, 7)])
def test_new_tree_graded_flags_followed_and_state_copied(params):
    T, u = _amr_case(42)
    flags, ni, nu = T.refine(u, *params)
    T2 = O.Tree(ni, T.bc)                  # raises if the new tree is not graded
    assert T2.lmin == T.lmin and T2.lmax <= params[2]
    old, new = _octs(T), _octs(T2)
    u2 = T2.permute_cells(nu)
    for key, o in old.items():
        i, j, k, l = key
        kept = key in new
        if l == T.lmin:
            assert kept
        else:
            f = old[(i >> 1, j >> 1, k >> 1, l - 1)]
            bit = (i & 1) + 2 * (j & 1) + 4 * (k & 1)
            assert kept == bool((flags[f] >> bit) & 1)
        if kept:
            # kept octs: children exactly where flagged, state unchanged
            assert int(T2.son_mask[new[key]]) == int(flags[o]), key
            assert np.array_equal(u2[8 * new[key]:8 * new[key] + 8], u[8 * o:8 * o + 8])
    # new octs: the father cell's values in all 8 cells
    for key, q in new.items():
        if key in old:
            continue
        i, j, k, l = key
        f = old[(i >> 1, j >> 1, k >> 1, l - 1)]
        src = u[8 * f + (i & 1) + 2 * (j & 1) + 4 * (k & 1)]
        assert np.array_equal(u2[8 * q:8 * q + 8], np.tile(src, (8, 1)))
    # the criterion's flags are a subset of the closed flags
    assert np.all((T.last_crit & ~flags) == 0)


@pytest.mark.parametrize("params", [(1.3, 0.0, 7), (0.0, 0.1, 6)])
def test_conservation(params):
    """Injection and removal of restricted children keep the leaf sums of
    volume * U (the removed octs' fathers hold their mean)."""
    T, u = _amr_case(43)
    _, ni, nu = T.refine(u, *params)
    T2 = O.Tree(ni, T.bc)
    u2 = T2.permute_cells(nu)
    a, abs_a = leaf_totals(T, u)
    b, abs_b = leaf_totals(T2, u2)
    assert np.all(np.abs(a - b) <= 1e-13 * np.maximum(abs_a, abs_b))


def test_closure_is_minimal():
    """Every split cell of the new tree whose children are leaves and which
    the criterion did not flag is needed: removing its child oct leaves the
    tree ungraded."""
    T, u = _amr_case(44)
    flags, ni, nu = T.refine(u, 1.35, 0.0, 6)
    T2 = O.Tree(ni, T.bc)
    old = _octs(T)
    checked = 0
    for q in range(T2.n):
        i, j, k, l = (int(v) for v in T2.ijkl[q])
        if l == T2.lmin or T2.son_mask[q]:
            continue
        fkey = (i >> 1, j >> 1, k >> 1, l - 1)
        bit = (i & 1) + 2 * (j & 1) + 4 * (k & 1)
        if (T.last_crit[old[fkey]] >> bit) & 1:
            continue
        rest = np.delete(T2.ijkl, q, axis=0)
        st, bad, *_ = O.neighbours(rest, T.bc)
        assert st == O.EUNGRADED, (i, j, k, l)
        checked += 1
    assert checked > 0


def _sphere_state(ijkl, centre, radius):
    cen, _ = I.cell_centres(ijkl)
    d = cen - np.asarray(centre)[None, None, :]
    d = d - np.round(d)
    inside = (d * d).sum(-1) < radius * radius
    z = np.zeros(cen.shape[:2])
    return I.conserved(np.where(inside, 2.0, 1.0), z, z, z, 1.0 + z, 1.4).reshape(-1, 5)


@pytest.mark.parametrize("start,centre,radius", [
    (lambda: I.uniform_tree(3), (0.4, 0.55, 0.5), 0.22),
    (lambda: I.sphere_tree(3, 6, (0.5, 0.5, 0.5), 0.3, I.PERIODIC), (0.3, 0.6, 0.45), 0.15),
])
def test_converges_to_the_static_sphere_tree(start, centre, radius):
    """With the density 2 inside a sphere and 1 outside (at every cell's
    centre) and rho_thresh 1.5, repeated refinement, growing or shrinking,
    stops at the tree the input module builds for that sphere, and stays."""
    lmax = 6
    ijkl = start()
    for it in range(2 * lmax):
        T = O.Tree(ijkl, I.PERIODIC)
        u = np.ascontiguousarray(_sphere_state(T.ijkl, centre, radius))
        _, ni, _ = T.refine(u, 1.5, 0.0, lmax)
        if len(ni) == T.n and set(map(tuple, ni.tolist())) == set(map(tuple, T.ijkl.tolist())):
            break
        ijkl = ni
    else:
        raise AssertionError("did not converge")
    want = O.Tree(I.sphere_tree(3, lmax, centre, radius, I.PERIODIC), I.PERIODIC)
    assert np.array_equal(want.keys, T.keys)


@pytest.mark.parametrize("params", [(1.3, 0.0, 7), (0.0, 0.1, 6)])
def test_block_refinement_keeps_sibling_groups(params):
    """nsubgrid = 4: octs above the coarsest level come in complete sibling
    groups (every split cell's oct is split in all 8 cells), the new tree is
    graded, the criterion's cells are split, and leaf sums are kept."""
    T, u = _amr_case(45)
    flags, ni, nu = T.refine(u, *params, nsubgrid=4)
    assert np.all((flags == 0) | (flags == 0xff))
    T2 = O.Tree(ni, T.bc)
    assert np.all((T2.son_mask == 0) | (T2.son_mask == 0xff))
    old, new = _octs(T), _octs(T2)
    for key, o in old.items():
        if key in new:
            assert int(T2.son_mask[new[key]]) == int(flags[o])
    # each removed oct leaves its father's restricted mean: one rounding each
    a, abs_a = leaf_totals(T, u)
    b, abs_b = leaf_totals(T2, T2.permute_cells(nu))
    assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(abs_a, abs_b))


def test_block_refinement_converges_to_the_static_block_tree():
    """Repeated block refinement on a sphere-shaped density reaches the
    block-structured sphere tree the input module builds independently."""
    centre, radius, lmax = (0.4, 0.55, 0.5), 0.22, 6
    ijkl = I.uniform_tree(3)
    for it in range(3 * lmax):
        T = O.Tree(ijkl, I.PERIODIC)
        u = np.ascontiguousarray(_sphere_state(T.ijkl, centre, radius))
        _, ni, _ = T.refine(u, 1.5, 0.0, lmax, nsubgrid=4)
        if len(ni) == T.n and set(map(tuple, ni.tolist())) == set(map(tuple, T.ijkl.tolist())):
            break
        ijkl = ni
    else:
        raise AssertionError("did not converge")
    want = O.Tree(I.sphere_tree(3, lmax, centre, radius, I.PERIODIC, blocks=True), I.PERIODIC)
    assert np.all((want.son_mask == 0) | (want.son_mask == 0xff))
    assert np.array_equal(want.keys, T.keys)
