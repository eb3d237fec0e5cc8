"""Pins of the oracle's multigrid Poisson solver (Sec. 5): the 7-point
Laplacian against its closed-form Fourier eigenvalues, the prolongation
against linear fields, red-black Gauss-Seidel as a convergent smoother, and
the V-cycle's residual reduction (the paper: about one order of magnitude
per cycle)."""
import numpy as np
import pytest

from oracle import oracle as O


def _grid(N):
    x = (np.arange(N) + 0.5) / N
    return np.meshgrid(x, x, x, indexing="ij")      # Z, Y, X


def _mode(N, k):
    Z, Y, X = _grid(N)
    f = np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z))
    h = 1.0 / N
    lam = sum((2 * np.cos(2 * np.pi * kk * h) - 2) / h ** 2 for kk in k)
    return f, f / lam


@pytest.mark.parametrize("k", [(1, 0, 0), (1, 2, 0), (3, 1, 2)])
def test_residual_vanishes_on_the_discrete_eigenfunction(k):
    f, phi = _mode(16, k)
    r = O.mg_residual(phi, f)
    assert np.abs(r).max() <= 1e-11 * np.abs(f).max()
    # and is f itself for phi = 0
    assert np.array_equal(O.mg_residual(np.zeros_like(f), f), f)


@pytest.mark.parametrize("k", [(1, 0, 0), (2, 1, 1), (3, 1, 2)])
def test_vcycles_reach_the_discrete_solution(k):
    f, want = _mode(32, k)
    phi, res = O.mg_vcycles(np.zeros_like(f), f, 12)
    phi = phi - phi.mean()
    assert np.abs(phi - want).max() <= 1e-9 * np.abs(want).max()


def test_one_order_of_magnitude_per_vcycle():
    rng = np.random.default_rng(5)
    N = 32
    f = rng.standard_normal((N, N, N))
    f -= f.mean()
    _, res = O.mg_vcycles(np.zeros_like(f), f, 8)
    rate = res[1:] / res[:-1]
    assert np.all(rate < 0.2), rate
    assert res[-1] < 1e-6 * res[0]


def test_prolongation_is_exact_for_linear_fields():
    """Trilinear interpolation from coarse centres reproduces a linear field
    at the fine centres wherever the stencil does not wrap around."""
    Nc = 8
    Zc, Yc, Xc = _grid(Nc)
    a = (0.7, -1.3, 2.1, 0.4)
    e = a[0] + a[1] * Xc + a[2] * Yc + a[3] * Zc
    phi = O.mg_prolong_add(e, np.zeros((2 * Nc,) * 3))
    Z, Y, X = _grid(2 * Nc)
    want = a[0] + a[1] * X + a[2] * Y + a[3] * Z
    inner = (slice(1, -1),) * 3
    assert np.abs(phi[inner] - want[inner]).max() <= 1e-14
    # a constant is reproduced everywhere (the weights sum to 64)
    one = O.mg_prolong_add(np.full((Nc,) * 3, 3.0), np.zeros((2 * Nc,) * 3))
    assert np.all(one == 3.0)


def test_gauss_seidel_converges_alone():
    """Red-black Gauss-Seidel on an 8^3 grid converges to the discrete
    solution by itself (slowly): the smoother is a consistent iteration."""
    f, want = _mode(8, (1, 1, 0))
    phi = O.mg_smooth(np.zeros_like(f), f, 400)
    phi = phi - phi.mean()
    assert np.abs(phi - want).max() <= 1e-8 * np.abs(want).max()
