"""Pins of the oracle's oct keys (Sec. 2.1 key tuple, Sec. 2.2 Hilbert order):
properties any correct 3-D Hilbert curve and the sentinel key layout must have."""
import numpy as np
import pytest

from oracle import oracle as O


def _grid(b):
    n = 1 << b
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], 1)


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5])
def test_bijection_and_unit_steps(b):
    """H_b is a bijection of the 2^b cube onto 0..8^b-1, and consecutive
    indices are face-adjacent cubes (the defining Hilbert property)."""
    pts = _grid(b)
    ijkl = np.concatenate([pts, np.full((len(pts), 1), b + 1)], 1).astype(np.int32)
    keys = O.keys(ijkl)
    h = keys - np.uint64(1 << (3 * b))
    assert np.array_equal(np.sort(h), np.arange(8 ** b, dtype=np.uint64))
    order = np.argsort(h)
    walk = pts[order]
    step = np.abs(np.diff(walk, axis=0)).sum(1)
    assert np.all(step == 1)


@pytest.mark.parametrize("b", [1, 2, 3, 4])
def test_nesting(b):
    """Children of the level-(b+1) oct (i,j,k) have keys 8K..8K+7 and
    key >> 3 gives the parent key."""
    pts = _grid(b)
    for i, j, k in pts[:: max(1, len(pts) // 64)]:
        K = O.key(i, j, k, b + 1)
        kids = sorted(O.key(2 * i + a, 2 * j + c, 2 * k + d, b + 2) for a in (0, 1) for c in (0, 1) for d in (0, 1))
        assert kids == list(range(8 * K, 8 * K + 8))
        for kk in kids:
            assert kk >> 3 == K


def test_key_layout_and_level_order():
    """Sentinel bit: keys of level l lie in [8^(l-1), 8^l); sorting keys sorts
    by level first; the single level-1 oct has key 1; no key is 0."""
    assert O.key(0, 0, 0, 1) == 1
    for l in range(1, 8):
        n = 1 << (l - 1)
        rng = np.random.default_rng(l)
        for _ in range(20):
            i, j, k = rng.integers(0, n, 3)
            K = O.key(i, j, k, l)
            assert (1 << (3 * (l - 1))) <= K < (1 << (3 * l))


def test_deep_levels_stay_consistent():
    """At deep levels the order-20 evaluation still nests and steps by one
    cube (sampled walk along a short stretch of level 13)."""
    l = 13
    b = l - 1
    rng = np.random.default_rng(7)
    for _ in range(30):
        i, j, k = (int(x) for x in rng.integers(0, 1 << b, 3))
        K = O.key(i, j, k, l)
        assert O.key(i >> 1, j >> 1, k >> 1, l - 1) == K >> 3
    # walk 512 consecutive level-13 keys inside one level-10 oct: unit steps
    base = O.key(5, 9, 3, 10) << 9
    pts = []
    lo = base
    par = (5 << 3, 9 << 3, 3 << 3)
    for di in range(8):
        for dj in range(8):
            for dk in range(8):
                pts.append((par[0] + di, par[1] + dj, par[2] + dk))
    pts = np.array(pts)
    ijkl = np.concatenate([pts, np.full((len(pts), 1), l)], 1).astype(np.int32)
    keys = O.keys(ijkl)
    assert np.array_equal(np.sort(keys), np.arange(lo, lo + 512, dtype=np.uint64))
    walk = pts[np.argsort(keys)]
    assert np.all(np.abs(np.diff(walk, axis=0)).sum(1) == 1)
