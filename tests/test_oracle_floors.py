"""Pins of the oracle's density and pressure floors (reading of the paper,
which states none: rho >= 1e-10 and p >= 1e-20 on primitive variables and on
the predicted face states) and of its OpenMP build.

- The floor counters see every kind of activation on a state built to
  need them, and the state stays finite with positive density; without the
  floors that state gives NaN (a planted missing floor fails here).
- On the Sod and Sedov configurations the floors never act, so the floor
  constants cannot change any result there.
- The OpenMP build of the same source gives the serial build's bits, for
  the global and the subcycled step, with injected and interpolated coarse
  ghosts, and the same floor counts."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2607_20704_amd import inputs as I


def test_prim_floor_values():
    O.floor_reset()
    W = O.prim(np.array([0.0, 0.0, 0.0, 0.0, 1.0]), 1.4)
    assert W[0] == 1e-10 and W[4] == (1.4 - 1.0) * 1.0
    W = O.prim(np.array([1.0, 10.0, 0.0, 0.0, 1.0]), 1.4)   # kinetic energy above E
    assert W[4] == 1e-20
    W = O.prim(np.array([1.0, 0.0, 0.0, 0.0, 1.0]), 1.4)
    assert W[0] == 1.0 and W[4] == (1.4 - 1.0) * 1.0
    assert O.floor_counts() == (1, 1, 0, 0)


def test_floor_stress_state():
    w = I.floor_stress()
    T = O.Tree(w.ijkl, w.bc)
    u = T.permute_cells(w.u)
    O.floor_reset()
    dts = T.run(u, w.gamma, w.cfl, w.nsteps)
    counts = O.floor_counts()
    assert all(c > 0 for c in counts), counts
    assert np.isfinite(u).all() and np.isfinite(dts).all()
    assert u[:, 0].min() > 0 and np.all(dts > 0)


def test_face_states_respect_floors():
    """Every predicted face state of every oct on the stressed state keeps
    rho >= 1e-10 and p >= 1e-20, while the counters show that the
    prediction alone would have gone below (so the bound is not vacuous)."""
    w = I.floor_stress()
    T = O.Tree(w.ijkl, w.bc)
    u = T.permute_cells(w.u)
    dt = T.cfl_dt(u, w.gamma, w.cfl)
    O.floor_reset()
    lo_rho, lo_p = np.inf, np.inf
    for o in range(T.n):
        S = T.face_states(u, o, dt, w.gamma)[:, :, 1:5, 1:5, 1:5, :]
        lo_rho = min(lo_rho, S[..., 0].min())
        lo_p = min(lo_p, S[..., 4].min())
    counts = O.floor_counts()
    assert counts[2] > 0 and counts[3] > 0, counts
    assert lo_rho >= 1e-10 and lo_p >= 1e-20, (lo_rho, lo_p)


@pytest.mark.parametrize("which", ["sod", "sedov"])
def test_floors_idle_on_benchmark_configs(which):
    w = I.sod_uniform() if which == "sod" else I.sedov_amr()
    T = O.Tree(w.ijkl, w.bc)
    u = T.permute_cells(w.u)
    with O.threads():
        O.floor_reset()
        T.run(u, w.gamma, w.cfl, w.nsteps)
        assert O.floor_counts() == (0, 0, 0, 0)


CASES = [
    ("amr_periodic_random", lambda: I.sphere_tree(3, 5, (0.4, 0.55, 0.5), 0.22, I.PERIODIC), I.PERIODIC),
    ("amr_outflow_random", lambda: I.sphere_tree(3, 5, (0.1, 0.2, 0.85), 0.25, I.OUTFLOW), I.OUTFLOW),
]


@pytest.mark.parametrize("name,mk,bc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("ghost", [O.GHOST_INJECT, O.GHOST_LINEAR])
def test_threaded_build_same_bits(name, mk, bc, ghost):
    ijkl = mk()
    gam = 5.0 / 3.0
    fields = I.random_fields_grid(8, 31, gamma=gam)
    u_in = I.grid_to_tree_state(ijkl, 3, fields, gam)
    T = O.Tree(ijkl, bc, ghost=ghost)
    a = T.permute_cells(u_in)
    b = a.copy()
    da = T.run(a, gam, 0.8, 4)
    sa = T.run_subcycled(a, gam, 0.8, 2)
    with O.threads():
        assert O.nthreads() >= 1
        db = T.run(b, gam, 0.8, 4)
        sb = T.run_subcycled(b, gam, 0.8, 2)
    assert np.array_equal(da, db) and np.array_equal(sa, sb)
    assert np.array_equal(a, b)


def test_threaded_floor_counts_match():
    w = I.floor_stress()
    T = O.Tree(w.ijkl, w.bc)
    a = T.permute_cells(w.u)
    b = a.copy()
    O.floor_reset()
    T.run(a, w.gamma, w.cfl, 3)
    serial = O.floor_counts()
    with O.threads():
        O.floor_reset()
        T.run(b, w.gamma, w.cfl, 3)
        threaded = O.floor_counts()
    assert np.array_equal(a, b) and serial == threaded
