"""GPU parity of the multigrid Poisson V-cycles (Sec. 5) against the
oracle's dense-grid V-cycles: residuals and whole cycles bit for bit, up to
the 256^3 unigrid the benchmark times, and the residual reduction per
cycle."""
import numpy as np
import pytest
import torch

from gpu_common import say
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _rhs(N, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((N, N, N))
    return f - f.mean()


def _to_dev(M, dense):
    ijk = M.fine_cells_ijk()
    return torch.as_tensor(np.ascontiguousarray(dense[ijk[:, 2], ijk[:, 1], ijk[:, 0]])).cuda()


def _to_dense(M, vals):
    ijk = M.fine_cells_ijk()
    N = 1 << M.lfine
    out = np.zeros((N, N, N))
    out[ijk[:, 2], ijk[:, 1], ijk[:, 0]] = vals.cpu().numpy()
    return out


def test_residual_bit_exact():
    from paper_2607_20704_amd import api
    M = api.Multigrid(5)
    N = 32
    phi, f = _rhs(N, 1), _rhs(N, 2)
    M.phi[M.fine] = _to_dev(M, phi)
    M.f[M.fine] = _to_dev(M, f)
    got = _to_dense(M, M.residual())
    assert np.array_equal(got, O.mg_residual(phi, f))


@pytest.mark.parametrize("lfine,lcoarse,nu,ncoarse,ncycles", [(5, 1, 2, 50, 3), (6, 2, 1, 20, 2), (4, 1, 3, 10, 4)])
def test_vcycles_bit_exact(lfine, lcoarse, nu, ncoarse, ncycles):
    from paper_2607_20704_amd import api
    M = api.Multigrid(lfine, lcoarse)
    N = 1 << lfine
    f = _rhs(N, 3 + lfine)
    M.f[M.fine] = _to_dev(M, f)
    M.vcycles(ncycles, nu, nu, ncoarse)
    torch.cuda.synchronize()
    want, res = O.mg_vcycles(np.zeros_like(f), f, ncycles, lcoarse, nu, nu, ncoarse)
    got = _to_dense(M, M.phi[M.fine])
    say("mg %d^3: max |diff| %.3g, residuals %s" % (N, np.abs(got - want).max(), res))
    assert np.array_equal(got, want)


def test_full_size_256_bit_exact_and_convergence():
    """The 256^3 unigrid of the benchmark: two V-cycles equal the oracle's,
    and the residual falls by about an order of magnitude per cycle."""
    from paper_2607_20704_amd import api
    M = api.Multigrid(8)
    N = 256
    f = _rhs(N, 11)
    M.f[M.fine] = _to_dev(M, f)
    r0 = float(torch.sqrt((M.residual() ** 2).mean()))
    M.vcycles(2)
    torch.cuda.synchronize()
    want, res = O.mg_vcycles(np.zeros_like(f), f, 2)
    got = _to_dense(M, M.phi[M.fine])
    assert np.array_equal(got, want)
    r2 = float(torch.sqrt((M.residual() ** 2).mean()))
    say("mg 256^3 residual %.3g -> %.3g (oracle %s)" % (r0, r2, res))
    assert abs(r2 - res[-1]) <= 1e-9 * res[-1]
    assert r2 < 0.02 * r0
