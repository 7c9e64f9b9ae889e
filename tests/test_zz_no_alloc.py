"""sap_solve_noalloc (static scratch, no allocation in the library) against
sap_create + sap_factor + sap_solve on the same options: identical results,
on two calls in a row, the second with a smaller input (the scratch keeps the
first call's contents, which must not leak into the second)."""

import numpy as np
import pytest
import torch

import sapgen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


CASES = [  # first call, then a smaller one
    dict(n=60000, k=20, p=32, mode="coupled", factor_prec="fp32", d=0.7),
    dict(n=9001, k=6, p=8, mode="decoupled", factor_prec="fp64", d=0.5),
]


def test_noalloc_matches_handle_path_twice():
    from paper_1509_07919_amd import SapSolver, sap
    for c in CASES:
        print("CASE noalloc", c, flush=True)
        n, k, p = c["n"], c["k"], c["p"]
        pb = sapgen.make_problem(n, k, d=c["d"], seed=48)
        a, b = dev(pb.band), dev(pb.b)
        opt = sap.make_options(n, k, p, c["mode"], c["factor_prec"])
        assert sap.sap_workspace_bytes(opt) + 256 <= sap.NOALLOC_SCRATCH_BYTES
        s = SapSolver(n, k, p, mode=c["mode"], factor_prec=c["factor_prec"], device=DEV)
        s.factor(a)
        x_ref, st_ref = s.solve(b, tol=1e-10, maxit=200)
        x, st = sap.solve_noalloc(a, b, n, k, p, mode=c["mode"], factor_prec=c["factor_prec"],
                                  tol=1e-10, maxit=200)
        torch.cuda.synchronize()
        assert st.status == sap.SAP_OK and st_ref.converged
        assert torch.equal(x, x_ref)
        assert (st.iters, st.restarts, st.n_apply, st.n_boosted) == \
            (st_ref.iters, st_ref.restarts, st_ref.n_apply, st_ref.n_boosted)
        assert st.rel_resid_true == st_ref.rel_resid_true <= 1e-10
        assert st.t_solve_ms == 0.0
        s.close()


def test_noalloc_rejects_options_beyond_the_scratch():
    from paper_1509_07919_amd import SapError, sap
    n, k, p = 200000, 50, 64
    opt = sap.make_options(n, k, p, "coupled", "fp64")
    assert sap.sap_workspace_bytes(opt) + 256 > sap.NOALLOC_SCRATCH_BYTES
    a = torch.zeros((2 * k + 1) * n, dtype=torch.float64, device=DEV)
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    with pytest.raises(SapError) as e:
        sap.solve_noalloc(a, b, n, k, p)
    assert e.value.code == sap.SAP_ERR_NOSPACE
    assert "static scratch holds" in str(e.value)
