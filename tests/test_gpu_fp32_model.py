"""FP32 factors at weak diagonal dominance, against an FP32 rounding-error
model evaluated by the oracle (Sec. 3.1 mixed precision: the preconditioner
runs in single precision).

The model (``oracle.dinv_error_sigma``): to first order the FP32 D^{-1}
returns g + A_i^{-1}(dr - E g), where the backward error E of the rounded
block, its LU and the two sweeps has entries of size u|A| + m u |L||U|
(m = 3K + 8 roundings per entry, u = 2^-24).  Treating the roundings as
independent with variance u^2/3 gives a standard deviation sigma per
component; the test allows 6 sigma (plus 8u|g|).  Worst-case signs
(``oracle.dinv_error_bound``) give a rigorous bound too, but at d = 0.12 it
exceeds max|g| and checks nothing.  The oracle pins both against an
independent float32 evaluation (tests/test_oracle_pins.py).

Chunked sweeps reassociate each block's sweep (chains over row chunks plus
a state recurrence through transfer matrices); with the state recurrence in
FP64 they meet the same model as one chain per block.  A solve with chunked
FP32 sweeps must also converge about as fast as with one chain per block.
"""

import numpy as np
import pytest
import torch

import oracle
import sapgen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solver(n, k, p, **kw):
    from paper_1509_07919_amd import SapSolver
    return SapSolver(n, k, p, device=DEV, **kw)


def check_model(z, M, r, blocks=None):
    sig = oracle.dinv_error_sigma(M, r, blocks=blocks)
    g = M.dinv(r)
    sel = ~np.isnan(sig)
    err = np.abs(z - g)[sel]
    lim = 6.0 * sig[sel] + 8 * U32 * np.abs(g[sel])
    worst = int(np.argmax(err / lim))
    assert np.all(err <= lim), "entry %d: error %.3e > 6 sigma %.3e (|g| %.3e)" % (
        np.flatnonzero(sel)[worst], err[worst], lim[worst], np.abs(g[sel][worst]))
    return float((err / np.maximum(sig[sel], 1e-300)).max())


@pytest.mark.parametrize("d", [0.5, 0.12])
@pytest.mark.parametrize("chunks", [1, 4])
def test_fp32_dinv_within_error_model(d, chunks):
    n, k, p = 6400, 24, 8
    print("CASE fp32-model", n, k, p, d, chunks, flush=True)
    pb = sapgen.make_problem(n, k, d=d, seed=47)
    M = oracle.SapPrecond(pb.band, n, k, p, False, boost_eps=2.0 ** -23)
    s = solver(n, k, p, mode="decoupled", factor_prec="fp32", sweep_chunks=chunks)
    s.factor(dev(pb.band))
    r = sapgen.splitmix64_uniform(8, 7, np.arange(n))
    ratio = check_model(host(s.precond(dev(r))), M, r)
    print("max |error| / sigma = %.2f" % ratio, flush=True)
    s.close()


@pytest.mark.parametrize("chunks", [1, 0])
def test_fp32_dinv_full_size_sampled_blocks(chunks):
    """N=200k, K=50, P=64 (the benchmark shape) at d = 0.11, where chunked
    FP32 chains once lost two orders of magnitude: the blocks with the
    largest chunk-state amplification are compared with the model."""
    n, k, p = 200000, 50, 64
    print("CASE fp32-model-full", chunks, flush=True)
    pb = sapgen.make_problem(n, k, d=0.11, seed=0)
    M = oracle.SapPrecond(pb.band, n, k, p, False, boost_eps=2.0 ** -23)
    s = solver(n, k, p, mode="decoupled", factor_prec="fp32", sweep_chunks=chunks)
    s.factor(dev(pb.band))
    r = sapgen.splitmix64_uniform(4, 7, np.arange(n))
    ratio = check_model(host(s.precond(dev(r))), M, r, blocks=[0, 25, 27, 38, 63])
    print("max |error| / sigma = %.2f" % ratio, flush=True)
    s.close()


def test_fp32_chunked_converges_like_one_chain():
    """Same system, same FP32 factors: the chunked sweeps (the default) may
    not slow BiCGStab(2) down by more than the spread that rounding alone
    causes at this dominance (at d ~ 0.1 a perturbation of 1e-15 in the
    preconditioner output moves an FP64 solve by +-10 %; FP32 evaluations in
    different orders differ by ~1e-4 and move it more): at most 1.6 times
    the iterations of one chain per block, plus one.  With the chunk states
    chained in FP32 the chunked solve took 24.75 iterations against 9.25."""
    n, k, p = 200000, 50, 64
    print("CASE fp32-chunked-iters", flush=True)
    pb = sapgen.make_problem(n, k, d=0.12, seed=0)
    a, b = dev(pb.band), dev(pb.b)
    its = {}
    for ch in (1, 0):
        s = solver(n, k, p, factor_prec="fp32", sweep_chunks=ch)
        s.factor(a)
        x, st = s.solve(b, tol=1e-10, maxit=200)
        assert st.converged
        assert np.abs(host(x) - pb.x_true).max() <= 1e-6 * np.abs(pb.x_true).max()
        its[ch] = st.iters
        s.close()
    print("iterations one chain %.2f, chunked %.2f" % (its[1], its[0]), flush=True)
    assert its[0] <= 1.6 * its[1] + 1.0
