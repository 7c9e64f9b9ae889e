"""Failure paths of the C ABI on the GPU, each forced from the host so that
every kernel still runs to its normal end:

* maxit too small: SAP_NOT_CONVERGED with the last iterate and its stats;
* an exact BiCGStab breakdown (gamma = 0), matched by the oracle;
* a non-finite right-hand side, reported as a breakdown;
* calls out of order.
The handle stays usable after each of them.
"""

import numpy as np
import pytest
import torch

import oracle
import sapgen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solver(n, k, p, **kw):
    from paper_1509_07919_amd import SapSolver
    return SapSolver(n, k, p, device=DEV, **kw)


def test_maxit_exhausted_returns_last_iterate():
    """SaP-D at d = 0.5 needs several iterations; with maxit = 1 the solve
    returns SAP_NOT_CONVERGED, x is the iterate after one BiCGStab(2)
    iteration and rel_resid_true is that iterate's true residual."""
    from paper_1509_07919_amd import SapError, sap
    n, k, p = 6000, 6, 12
    print("CASE maxit", n, k, p, flush=True)
    pb = sapgen.make_problem(n, k, d=0.5, seed=41)
    s = solver(n, k, p, mode="decoupled", factor_prec="fp64")
    s.factor(dev(pb.band))
    x, st = s.solve(dev(pb.b), tol=1e-12, maxit=1)
    assert st.status == sap.SAP_NOT_CONVERGED and not st.converged
    assert st.iters == 1.0 and st.n_apply == 4 and st.restarts == 0
    xh = host(x)
    assert np.all(np.isfinite(xh))
    res = np.linalg.norm(pb.b - oracle.bandmv(pb.band, n, k, xh)) / np.linalg.norm(pb.b)
    assert abs(res - st.rel_resid_true) <= 1e-12 + 1e-9 * res
    assert 1e-12 < st.rel_resid_true < 1.0
    # the oracle's iterate after one iteration is the same vector
    ref = oracle.bicgstab_l(lambda v: oracle.bandmv(pb.band, n, k, v),
                            oracle.SapPrecond(pb.band, n, k, p, False).apply,
                            pb.b, tol=1e-12, maxit=1)
    assert not ref.converged and ref.iters == 1.0
    assert np.abs(xh - ref.x).max() <= 1e-9 * np.abs(ref.x).max()
    with pytest.raises(SapError) as e:
        s.solve(dev(pb.b), tol=1e-12, maxit=1, raise_nc=True)
    assert e.value.code == sap.SAP_NOT_CONVERGED
    x2, st2 = s.solve(dev(pb.b), tol=1e-10, maxit=200)       # still usable
    assert st2.converged
    s.close()


def zero_row_sum_problem(n):
    """K = 1, unit diagonal, off-diagonals -1/2 (-1 in the two end rows): every
    row sums to exactly zero, so A 1 = 0 in floating point."""
    k = 1
    band = np.zeros(3 * n)
    band[n:2 * n] = 1.0                                    # diagonal
    band[1:n] = -0.5                                       # a[c-1][c] at q = 0
    band[1] = -1.0                                         # a[0][1]
    band[2 * n:3 * n - 1] = -0.5                           # a[c+1][c] at q = 2
    band[3 * n - 2] = -1.0                                 # a[n-1][n-2]
    return band, k


def test_exact_breakdown_gamma_zero():
    """SaP-D with 1x1 blocks on the zero-row-sum matrix: M = diag(A) = I, so
    with b = 1 the first BiCG step gives u1 = M^{-1} A 1 = 0 exactly and
    gamma = (u1, r~) = 0: a true breakdown of BiCGStab.  The library returns
    SAP_ERR_BREAKDOWN, as the oracle raises Breakdown."""
    from paper_1509_07919_amd import SapError, sap
    n = 64
    print("CASE breakdown", n, flush=True)
    band, k = zero_row_sum_problem(n)
    assert np.array_equal(oracle.bandmv(band, n, k, np.ones(n)), np.zeros(n))
    with pytest.raises(oracle.Breakdown):
        oracle.bicgstab_l(lambda v: oracle.bandmv(band, n, k, v),
                          oracle.SapPrecond(band, n, k, n, False).apply, np.ones(n))
    s = solver(n, k, n, mode="decoupled", factor_prec="fp64")
    s.factor(dev(band))
    with pytest.raises(SapError) as e:
        s.solve(dev(np.ones(n)), tol=1e-10, maxit=10)
    assert e.value.code == sap.SAP_ERR_BREAKDOWN
    # a consistent right-hand side on a nonsingular matrix still solves
    band2 = band.copy()
    band2[n:2 * n] = 4.0
    xt = sapgen.splitmix64_uniform(42, 2, np.arange(n))
    b2 = oracle.bandmv(band2, n, k, xt)
    s.factor(dev(band2))
    x2, st2 = s.solve(dev(b2), tol=1e-12, maxit=200)
    assert st2.converged
    assert np.abs(host(x2) - xt).max() <= 1e-10
    s.close()


def test_non_finite_rhs_is_a_breakdown():
    from paper_1509_07919_amd import SapError, sap
    n, k, p = 3000, 5, 6
    print("CASE nan-rhs", n, k, p, flush=True)
    pb = sapgen.make_problem(n, k, seed=43)
    s = solver(n, k, p, factor_prec="fp32")
    s.factor(dev(pb.band))
    b = pb.b.copy()
    b[1234] = np.nan
    with pytest.raises(SapError) as e:
        s.solve(dev(b), tol=1e-10, maxit=10)
    assert e.value.code == sap.SAP_ERR_BREAKDOWN
    x, st = s.solve(dev(pb.b), tol=1e-10, maxit=100)
    assert st.converged
    assert np.abs(host(x) - pb.x_true).max() <= 1e-8
    s.close()


def test_calls_out_of_order():
    from paper_1509_07919_amd import SapError, sap
    n, k, p = 1000, 3, 4
    print("CASE order", n, k, p, flush=True)
    s = solver(n, k, p, factor_prec="fp64")
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    with pytest.raises(SapError) as e:
        s.solve(b)
    assert e.value.code == sap.SAP_ERR_STATE
    pb = sapgen.make_problem(n, k, seed=44)
    s.factor(dev(pb.band))
    with pytest.raises(SapError) as e:                      # created without adjoint
        s.solve_adjoint(b)
    assert e.value.code == sap.SAP_ERR_STATE
    s.close()
