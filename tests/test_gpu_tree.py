"""GPU parity of the integer path (keys, radix sort, level ranges, FNV hash,
neighbour lists) against the oracle: bit-exact."""
import numpy as np
import pytest
import torch

from gpu_common import build_both, say, small_trees
from oracle import oracle as O
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_keys_match_oracle_random_deep():
    from paper_2607_20704_amd import api
    rng = np.random.default_rng(9)
    rows = []
    for l in range(1, 22):
        n = 1 << (l - 1)
        for _ in range(300):
            rows.append([*rng.integers(0, n, 3), l])
    ijkl = np.array(rows, np.int32)
    say("keys: %d random octs on levels 1..21" % len(ijkl))
    keys = api.encode_keys(torch.as_tensor(ijkl).cuda()).cpu().numpy()
    assert np.array_equal(keys, O.keys(ijkl))
    back = api.decode_keys(torch.as_tensor(keys.astype(np.int64)).cuda().view(torch.uint64)).cpu().numpy()
    assert np.array_equal(back, ijkl)


@pytest.mark.parametrize("name", ["sod_l5", "sedov_l6_l8", "uniform_l8"])
def test_sort_and_level_ranges(name):
    from paper_2607_20704_amd import api
    ijkl = {"sod_l5": lambda: I.uniform_tree(5), "sedov_l6_l8": lambda: I.sedov_amr().ijkl,
            "uniform_l8": lambda: I.uniform_tree(8)}[name]()
    # shuffle the input so the sort has work to do
    ijkl = ijkl[np.random.default_rng(1).permutation(len(ijkl))]
    say("sort: %s, %d octs" % (name, len(ijkl)))
    keys = api.encode_keys(torch.as_tensor(ijkl).cuda())
    skeys, perm = api.sort_keys(keys)
    assert np.array_equal(perm.cpu().numpy(), O.tree_order(ijkl))
    sk = skeys.cpu().numpy()
    assert np.array_equal(sk, np.sort(O.keys(ijkl)))
    begin = api.level_ranges(skeys).cpu().numpy()
    lv = ijkl[:, 3]
    for l in range(0, 23):
        assert begin[l] == np.count_nonzero(lv < l), l


def test_hash_lookup_and_errors():
    from paper_2607_20704_amd import api
    from paper_2607_20704_amd import _lib as L
    ijkl = I.sedov_amr().ijkl
    say("hash: sedov tree, %d keys" % len(ijkl))
    keys = torch.as_tensor(O.keys(ijkl).astype(np.int64)).cuda().view(torch.uint64)
    ws = api.hash_build(keys)
    assert api.check_ws(ws) == (L.RG_OK, -1)
    idx = api.hash_lookup(ws, keys).cpu().numpy()
    assert np.array_equal(idx, np.arange(len(ijkl)))
    # absent keys: children of the finest level, and key 0
    absent = O.keys(np.concatenate([2 * ijkl[-50:, :3], ijkl[-50:, 3:] + 1], 1))
    q = torch.as_tensor(np.concatenate([absent, [0]]).astype(np.int64)).cuda().view(torch.uint64)
    assert np.all(api.hash_lookup(ws, q).cpu().numpy() == -1)
    # duplicate key
    hk = O.keys(ijkl).astype(np.int64)
    dup = torch.as_tensor(np.concatenate([hk[:100], hk[:1]])).cuda().view(torch.uint64)
    ws2 = api.hash_build(dup)
    st, bad = api.check_ws(ws2)
    assert st == L.RG_EDUPKEY and bad in (0, 100)
    # zero key
    z = hk[:10].copy()
    z[3] = 0
    ws3 = api.hash_build(torch.as_tensor(z).cuda().view(torch.uint64))
    assert api.check_ws(ws3) == (L.RG_EINVAL, 3)


@pytest.mark.parametrize("case", small_trees(), ids=[c[0] for c in small_trees()])
def test_neighbours_match_oracle(case):
    name, ijkl, bc, _ = case
    say("neighbours:", name, len(ijkl))
    T, D = build_both(ijkl, bc)
    check_lists(T, D)


def check_lists(T, D):
    """Lists of the plain build, then of the scheduled (brick-local) rebuild
    after re-keying, all equal to the oracle's."""
    from paper_2607_20704_amd import api
    assert np.array_equal(D.nbr27.cpu().numpy(), T.nbr27)
    assert np.array_equal(D.father_cell.cpu().numpy(), T.father_cell)
    assert np.array_equal(D.son_mask.cpu().numpy(), T.son_mask.astype(np.int32))
    say("  schedule", D.schedule_counts(), "bricks for lists", D.sched.nbr_brick_count,
        "other octs", D.sched.nbr_rest_count)
    D.nbr27.fill_(-7)
    D.father_cell.fill_(-7)
    D.son_mask.fill_(-7)
    D.prepare()
    assert api.check_ws(D.hash_ws)[0] == 0
    assert np.array_equal(D.keys.cpu().numpy(), T.keys)
    assert np.array_equal(D.perm_scratch.cpu().numpy(), np.arange(T.n))
    assert np.array_equal(D.level_begin_dev.cpu().numpy(), D.level_begin)
    assert np.array_equal(D.nbr27.cpu().numpy(), T.nbr27)
    assert np.array_equal(D.father_cell.cpu().numpy(), T.father_cell)
    assert np.array_equal(D.son_mask.cpu().numpy(), T.son_mask.astype(np.int32))


@pytest.mark.parametrize("name", ["sedov_l6_l8", "uniform_l8_periodic", "uniform_l5_outflow", "sedov_l4_l6"])
def test_neighbours_match_oracle_large(name):
    w = {"sedov_l6_l8": lambda: (I.sedov_amr().ijkl, I.PERIODIC),
         "uniform_l8_periodic": lambda: (I.uniform_tree(8), I.PERIODIC),
         "uniform_l5_outflow": lambda: (I.uniform_tree(5), I.OUTFLOW),
         "sedov_l4_l6": lambda: (I.sedov_amr(base=4, lmax=6).ijkl, I.PERIODIC)}[name]
    ijkl, bc = w()
    say("neighbours:", name, len(ijkl))
    T, D = build_both(ijkl, bc)
    check_lists(T, D)


def test_ungraded_tree_is_reported():
    from paper_2607_20704_amd import api
    from paper_2607_20704_amd import _lib as L
    base = I.uniform_tree(2)
    tree = np.concatenate([base, [[2, 2, 2, 3]], [[4, 4, 4, 4]]]).astype(np.int32)
    perm = O.tree_order(tree)
    st_o, bad_o, *_ = O.neighbours(tree[perm], I.PERIODIC)
    say("ungraded tree, %d octs" % len(tree))
    keys = torch.as_tensor(O.keys(tree[perm]).astype(np.int64)).cuda().view(torch.uint64)
    ws = api.hash_build(keys)
    api.build_neighbours(ws, keys, 2, I.PERIODIC)
    st, bad = api.check_ws(ws)
    assert st == L.RG_EUNGRADED == st_o
    assert bad == bad_o


def _fnv1a64_np(k):
    """FNV-1a 64 over the 8 little-endian bytes, vectorised (uint64 wraps)."""
    h = np.full(k.shape, 0xCBF29CE484222325, dtype=np.uint64)
    for b in range(8):
        h ^= (k >> np.uint64(8 * b)) & np.uint64(0xFF)
        h *= np.uint64(0x100000001B3)
    return h


def test_hash_build_probe_runs_leave_their_segment():
    """Keys chosen so that many home slots fall at the end of 4096-slot
    segments (and at the end of the table, where probing wraps to slot 0):
    the probe sequences leave their segment and are finished on the whole
    table.  Every key is found at its index, absent keys are not, and a
    duplicate among them is reported."""
    from paper_2607_20704_amd import api
    from paper_2607_20704_amd import _lib as L
    n = 6000
    cap = 16384
    rng = np.random.default_rng(5)
    cand = np.unique(rng.integers(1, 2 ** 63, 4_000_000, dtype=np.int64).astype(np.uint64))
    assert L.lib().rg_fnv1a64(int(cand[0])) == int(_fnv1a64_np(cand[:1])[0])
    home = _fnv1a64_np(cand) & np.uint64(cap - 1)
    # 40 keys on each of the last 8 slots of every segment, then random keys
    aimed = []
    for slot in [s0 + j for s0 in range(4095, cap, 4096) for j in range(-7, 1)]:
        aimed.append(cand[home == np.uint64(slot)][:40])
    aimed = np.concatenate(aimed)
    assert len(aimed) == 4 * 8 * 40
    rest = np.setdiff1d(cand, aimed)
    chosen = np.concatenate([aimed, rng.permutation(rest)[:n - len(aimed)]])
    keys_np = rng.permutation(chosen)
    seen = set(int(k) for k in keys_np)
    say("hash overflow: %d keys, %d aimed at segment ends" % (n, 4 * 8 * 40))
    keys = torch.as_tensor(keys_np.view(np.int64)).cuda().view(torch.uint64)
    ws = api.hash_build(keys)
    assert api.check_ws(ws) == (L.RG_OK, -1)
    assert np.array_equal(api.hash_lookup(ws, keys).cpu().numpy(), np.arange(n))
    absent = np.array([int(k) for k in rest[-2000:] if int(k) not in seen][:500], dtype=np.uint64)
    q = torch.as_tensor(absent.view(np.int64)).cuda().view(torch.uint64)
    assert np.all(api.hash_lookup(ws, q).cpu().numpy() == -1)
    # a duplicate of a key whose home is at a segment end
    first = int(np.nonzero(np.isin(keys_np, aimed))[0][0])
    dup = np.concatenate([keys_np, keys_np[first:first + 1]])
    ws2 = api.hash_build(torch.as_tensor(dup.view(np.int64)).cuda().view(torch.uint64))
    st, bad = api.check_ws(ws2)
    assert st == L.RG_EDUPKEY and bad in (first, n)


def test_empty_inputs():
    """Zero counts and empty oct ranges return RG_OK and write nothing; an
    empty hash table answers -1; the time step over no octs is +inf."""
    from paper_2607_20704_amd import api
    say("empty inputs")
    ijkl = torch.empty((0, 4), dtype=torch.int32, device="cuda")
    keys = api.encode_keys(ijkl)
    assert keys.shape == (0,)
    assert api.decode_keys(keys).shape == (0, 4)
    skeys, perm = api.sort_keys(keys)
    assert skeys.shape == (0,) and perm.shape == (0,)
    assert not api.level_ranges(skeys).cpu().numpy().any()
    ws = api.hash_build(keys)
    assert api.check_ws(ws) == (0, -1)
    q = torch.as_tensor(O.keys(I.uniform_tree(2)).astype(np.int64)).cuda().view(torch.uint64)
    assert np.all(api.hash_lookup(ws, q).cpu().numpy() == -1)
    assert api.hash_lookup(ws, keys).shape == (0,)
    nbr27, father, son = api.build_neighbours(ws, keys, 1, api.RG_BC_PERIODIC)
    assert nbr27.shape == (0, 27) and father.shape == (0,) and son.shape == (0,)
    x = torch.empty((0, 5), dtype=torch.float64, device="cuda")
    assert api.permute_rows(x, perm).shape == (0, 5)
    # empty oct ranges: no pointer is read, nothing is written
    for form in (api.RG_FP64, api.RG_MIXED):
        api.hydro_step_level(0.5, None, 1.4, None, None, None, None, 3, 3, form=form)
    api.apply_coarse_corrections(None, None, 0, None, 5, 5)
    api.restrict_level(None, None, 7, 7)
    u = torch.full((16, 5), 7.0, dtype=torch.float64, device="cuda")
    un = u.clone()
    dt = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    nb = torch.zeros((2, 27), dtype=torch.int32, device="cuda")
    sm = torch.zeros(2, dtype=torch.int32, device="cuda")
    api.hydro_step_level(0.5, dt, 1.4, u, un, nb, sm, 1, 1, cfl=0.8, dt_next=dt)
    torch.cuda.synchronize()
    assert torch.equal(un, u) and dt.item() == 0.25
    # the time step over levels that hold no octs
    d = api.cfl_dt(u, sm, np.zeros(api.RG_MAX_LEVEL + 2, np.int64), 1, 3, 1.4, 0.8)
    assert d.item() == float("inf")


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9])
def test_hash_tiny_tables(n):
    """Tables below one segment (capacity 16 and 32): every key found at its
    index, absent keys answer -1."""
    from paper_2607_20704_amd import api
    from paper_2607_20704_amd import _lib as L
    hk = O.keys(I.uniform_tree(3)).astype(np.int64)
    say("hash: %d keys" % n)
    sel = hk[np.random.default_rng(n).permutation(len(hk))[:n]]
    keys = torch.as_tensor(sel).cuda().view(torch.uint64)
    ws = api.hash_build(keys)
    assert api.check_ws(ws) == (L.RG_OK, -1)
    assert np.array_equal(api.hash_lookup(ws, keys).cpu().numpy(), np.arange(n))
    rest = torch.as_tensor(np.setdiff1d(hk, sel)).cuda().view(torch.uint64)
    assert np.all(api.hash_lookup(ws, rest).cpu().numpy() == -1)
