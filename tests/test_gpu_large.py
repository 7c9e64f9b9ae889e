"""A system whose band holds more than 2^31 entries ((2K+1) N = 2.17e9 at
N = 21.5M, K = 50: every index into A, the factors and the vectors must be
64-bit).  Too large for the oracle, so the checks are properties that hold
at any size: the solution against x_true, and the true residual
||b - A x|| / ||b||, both evaluated with plain PyTorch operations on the
band (one shifted slice per diagonal), independent of the library's kernels.

The matrix is built on the GPU: off-diagonal entries uniform in [-1, 1)
from a seeded torch generator, the diagonal 1.5 times the row's absolute
sum (strictly dominant, as the dense workloads with d = 1.5).
"""

import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def band_matvec(band, n, k, x):
    """y = A x for A in band layout (band[q*n + c] = a[c + q - K][c])."""
    b2 = band.view(2 * k + 1, n)
    y = torch.zeros(n, dtype=torch.float64, device=band.device)
    for q in range(2 * k + 1):
        d = q - k                              # row = col + d
        if d >= 0:
            y[d:] += b2[q, :n - d] * x[:n - d]
        else:
            y[:n + d] += b2[q, -d:] * x[-d:]
    return y


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_band_beyond_2_31_entries(prec):
    from paper_1509_07919_amd import SapSolver
    n, k, p = 21_500_000, 50, 2048
    assert (2 * k + 1) * n > 2 ** 31
    print("CASE large", n, k, p, prec, flush=True)
    g = torch.Generator(device=DEV)
    g.manual_seed(1234)
    band = torch.rand((2 * k + 1) * n, dtype=torch.float64, device=DEV, generator=g) * 2.0 - 1.0
    b2 = band.view(2 * k + 1, n)
    # zero the slots outside the matrix, then the diagonal from the row sums
    for q in range(2 * k + 1):
        d = q - k
        if d > 0:
            b2[q, n - d:] = 0.0
        elif d < 0:
            b2[q, :-d] = 0.0
    b2[k].zero_()
    rowsum = band_matvec(band.abs(), n, k, torch.ones(n, dtype=torch.float64, device=DEV))
    b2[k] = 1.5 * rowsum
    del rowsum
    x_true = torch.rand(n, dtype=torch.float64, device=DEV, generator=g) * 2.0 - 1.0
    rhs = band_matvec(band, n, k, x_true)
    s = SapSolver(n, k, p, mode="coupled", factor_prec=prec, device=DEV)
    s.factor(band)
    x, st = s.solve(rhs, tol=1e-10, maxit=200)
    torch.cuda.synchronize()
    assert st.converged, st
    err = float(torch.linalg.norm(x - x_true) / torch.linalg.norm(x_true))
    res = float(torch.linalg.norm(rhs - band_matvec(band, n, k, x)) / torch.linalg.norm(rhs))
    print("large", prec, "iters", st.iters, "err", err, "res", res, flush=True)
    assert err <= 1e-8
    assert res <= 1e-10 * 1.001
    s.close()
    del band, x_true, rhs, x
    torch.cuda.empty_cache()
