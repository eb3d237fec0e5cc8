"""Pins of the oracle's per-cell and per-face pieces (Sec. 3: primitive
variables, minmod reconstruction, HLLC Riemann flux) by exact identities."""
import numpy as np
import pytest

from oracle import oracle as O

GAMMAS = [1.4, 5.0 / 3.0]


def euler_flux(W, axis, gamma):
    """Physical flux of the Euler equations, written out from its definition."""
    rho, u, v, w, p = W
    vel = np.array([u, v, w])
    un = vel[axis]
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    F = np.empty(5)
    F[0] = rho * un
    F[1:4] = rho * un * vel
    F[1 + axis] += p
    F[4] = (E + p) * un
    return F


def rand_state(rng, vmax=2.0):
    return np.array([rng.uniform(0.1, 3.0), *rng.uniform(-vmax, vmax, 3), rng.uniform(0.05, 4.0)])


@pytest.mark.parametrize("gamma", GAMMAS)
def test_prim_round_trip(gamma):
    rng = np.random.default_rng(1)
    for _ in range(200):
        W = rand_state(rng)
        rho, u, v, w, p = W
        U = np.array([rho, rho * u, rho * v, rho * w, p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)])
        W2 = O.prim(U, gamma)
        assert np.allclose(W2, W, rtol=1e-13, atol=1e-14 * np.abs(W).max())


def test_prim_floors():
    W = O.prim(np.array([-1.0, 0.0, 0.0, 0.0, 1.0]), 1.4)
    assert W[0] == 1e-10
    W = O.prim(np.array([1.0, 10.0, 0.0, 0.0, 1.0]), 1.4)   # kinetic energy exceeds E
    assert W[4] == 1e-20


def primitive_jacobians(W, gamma):
    """A_x, A_y, A_z of the primitive Euler system W_t + sum_d A_d W_d = 0,
    W = (rho, u, v, w, p), written out from the equations
    rho_t + u.grad rho + rho div u = 0, u_t + u.grad u + grad p / rho = 0,
    p_t + u.grad p + gamma p div u = 0."""
    rho, u, v, w, p = W
    vel = (u, v, w)
    As = []
    for d in range(3):
        A = np.diag([vel[d]] * 5).astype(float)
        A[0, 1 + d] = rho
        A[1 + d, 4] = 1.0 / rho
        A[4, 1 + d] = gamma * p
        As.append(A)
    return As


@pytest.mark.parametrize("gamma", GAMMAS)
def test_predictor_is_half_step_of_primitive_equations(gamma):
    rng = np.random.default_rng(3)
    for _ in range(300):
        W = rand_state(rng)
        dW = rng.normal(size=(3, 5)) * 0.1
        h = rng.uniform(0.01, 0.5)
        want = W - h * sum(A @ dW[d] for d, A in enumerate(primitive_jacobians(W, gamma)))
        got = O.predict(W, dW, h, gamma)
        assert np.allclose(got, want, rtol=1e-14, atol=1e-14 * np.abs(W).max())


def test_minmod_cases():
    cases = [((1.0, 2.0), 1.0), ((2.0, 1.0), 1.0), ((-1.0, -3.0), -1.0), ((-3.0, -1.0), -1.0),
             ((1.0, -1.0), 0.0), ((-1.0, 1.0), 0.0), ((0.0, 1.0), 0.0), ((1.0, 0.0), 0.0), ((0.0, 0.0), 0.0)]
    for (a, b), want in cases:
        assert O.minmod(a, b) == want


@pytest.mark.parametrize("gamma", GAMMAS)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_consistency(gamma, axis):
    """F(W, W) is the physical flux."""
    rng = np.random.default_rng(2 + axis)
    for _ in range(200):
        W = rand_state(rng)
        F = O.hllc(W, W, axis, gamma)
        Fe = euler_flux(W, axis, gamma)
        scale = np.abs(Fe).max() + W[4]
        assert np.all(np.abs(F - Fe) <= 8e-16 * 4 * scale)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_stationary_contact(axis):
    """A contact at rest with equal pressure carries no mass, transverse
    momentum or energy; the normal momentum flux is the pressure."""
    rng = np.random.default_rng(10 + axis)
    for _ in range(100):
        p = rng.uniform(0.1, 3.0)
        WL = np.array([rng.uniform(0.1, 3), 0, 0, 0, p])
        WR = np.array([rng.uniform(0.1, 3), 0, 0, 0, p])
        for a in range(3):
            if a != axis:
                WL[1 + a] = rng.uniform(-1, 1)
                WR[1 + a] = rng.uniform(-1, 1)
        F = O.hllc(WL, WR, axis, 1.4)
        assert F[0] == 0.0 and F[4] == 0.0
        for a in range(3):
            if a != axis:
                assert F[1 + a] == 0.0
        assert abs(F[1 + axis] - p) <= 4e-16 * p


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_mirror_antisymmetry(axis):
    """Exchanging the sides and reversing the normal velocity reverses mass,
    energy and transverse momentum fluxes and keeps the normal momentum flux,
    bit for bit (the star state is written in a side-symmetric form)."""
    rng = np.random.default_rng(20 + axis)
    for _ in range(500):
        WL, WR = rand_state(rng), rand_state(rng)
        F = O.hllc(WL, WR, axis, 1.4)
        ML, MR = WR.copy(), WL.copy()
        ML[1 + axis] *= -1
        MR[1 + axis] *= -1
        G = O.hllc(ML, MR, axis, 1.4)
        sign = -np.ones(5)
        sign[1 + axis] = 1
        assert np.array_equal(G, sign * F)


def test_hllc_supersonic_upwind():
    """All waves moving right: the flux is the left physical flux, exactly."""
    WL = np.array([1.0, 5.0, 0.3, -0.2, 1.0])
    WR = np.array([0.5, 4.0, 0.1, 0.2, 0.8])
    F = O.hllc(WL, WR, 0, 1.4)
    assert np.array_equal(F, O.hllc(WL, WL, 0, 1.4))
    WL2, WR2 = WR.copy(), WL.copy()
    WL2[1], WR2[1] = -4.0, -5.0
    F2 = O.hllc(WL2, WR2, 0, 1.4)
    assert np.array_equal(F2, O.hllc(WR2, WR2, 0, 1.4))


def toro_hllc(WL, WR, axis, gamma):
    """HLLC as printed in Toro (2009) sec. 10.4: Davis speeds, S* from his
    eq. 10.37, star states from eq. 10.39, F*_K = F_K + S_K (U*_K - U_K)."""
    def cons(W):
        rho, u, v, w, p = W
        return np.array([rho, rho * u, rho * v, rho * w, p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)])
    rl, pl, ul = WL[0], WL[4], WL[1 + axis]
    rr, pr, ur = WR[0], WR[4], WR[1 + axis]
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    SL, SR = min(ul - cl, ur - cr), max(ul + cl, ur + cr)
    Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))
    if SL > 0:
        return euler_flux(WL, axis, gamma)
    if SR <= 0:
        return euler_flux(WR, axis, gamma)
    W, S = (WL, SL) if Ss > 0 else (WR, SR)
    U = cons(W)
    rho, un, p = W[0], W[1 + axis], W[4]
    fac = rho * (S - un) / (S - Ss)
    Us = fac * np.array([1.0, *W[1:4], U[4] / rho + (Ss - un) * (Ss + p / (rho * (S - un)))])
    Us[1 + axis] = fac * Ss
    return euler_flux(W, axis, gamma) + S * (Us - U)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_equals_textbook_form(axis):
    """The side-symmetric S*/p* and the direct F(U*) agree with Toro's printed
    HLLC to rounding, in all four wave regions."""
    rng = np.random.default_rng(30 + axis)
    regions = set()
    for _ in range(2000):
        WL, WR = rand_state(rng, vmax=4.0), rand_state(rng, vmax=4.0)
        F = O.hllc(WL, WR, axis, 1.4)
        T = toro_hllc(WL, WR, axis, 1.4)
        scale = np.abs(T).max() + max(WL[4], WR[4])
        assert np.all(np.abs(F - T) <= 1e-12 * scale)
        ul, ur = WL[1 + axis], WR[1 + axis]
        SL = min(ul - np.sqrt(1.4 * WL[4] / WL[0]), ur - np.sqrt(1.4 * WR[4] / WR[0]))
        SR = max(ul + np.sqrt(1.4 * WL[4] / WL[0]), ur + np.sqrt(1.4 * WR[4] / WR[0]))
        regions.add((SL > 0, SR > 0))
    assert len(regions) == 3
