"""Sparse front end on the host (no GPU): the library's diagonal boosting,
Cuthill-McKee and drop-off against the oracle (oracle/sparse.py), and the
oracle's matching against brute force."""

import itertools

import numpy as np
import pytest

import oracle.sparse as osp
import sapgen


@pytest.fixture(scope="module")
def lib():
    from paper_1509_07919_amd import sap
    return sap.load_library()


def plan(sp, db=True, cm=True, drop=0.0):
    from paper_1509_07919_amd import SapSparse
    return SapSparse(sp.n, sp.rowptr, sp.colidx, sp.vals, db=db, cm=cm, drop_frac=drop)


@pytest.mark.parametrize("n", [3, 5, 7, 8])
def test_oracle_matching_is_the_brute_force_optimum(n):
    """min over all permutations of sum c_{i sigma_i} (eq:DBrelated)."""
    rng_u = sapgen.splitmix64_uniform(70 + n, 6, np.arange(n * n)).reshape(n, n)
    A = np.where(np.abs(rng_u) < 0.6, rng_u, 0.0) + np.eye(n)[::-1] * 0.05
    rows, cols = np.nonzero(A)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))])
    sigma, cost = osp.db_matching(n, rowptr, cols, A[rows, cols])
    amax = np.abs(A).max(axis=1)
    best = min(sum(np.log(amax[i]) - np.log(abs(A[i, p[i]])) if A[i, p[i]] != 0 else np.inf
                   for i in range(n)) for p in itertools.permutations(range(n)))
    assert abs(cost - best) <= 1e-12
    assert sorted(sigma) == list(range(n))


@pytest.mark.parametrize("n,k0,density,seed", [(500, 4, 0.5, 1), (3000, 10, 0.3, 2),
                                               (4000, 25, 0.15, 3)])
def test_db_matching_cost_and_i_matrix(n, k0, density, seed):
    sp = sapgen.make_sparse_problem(n, k0, density=density, seed=seed)
    info = plan(sp, db=True, cm=False).info()
    sigma = info["new_row"]
    assert sorted(sigma) == list(range(n))
    cost = osp.matching_cost(n, sp.rowptr, sp.colidx, sp.vals, sigma)
    sigma_o, best = osp.db_matching(n, sp.rowptr, sp.colidx, sp.vals)
    assert abs(cost - best) <= 1e-9 * max(1.0, abs(best))
    # continuous random values: the optimum is unique, so the matchings agree
    assert np.array_equal(sigma, sigma_o)
    sigma_s, cost_s = osp.db_matching_scipy(n, sp.rowptr, sp.colidx, sp.vals)
    assert np.array_equal(sigma_o, sigma_s) and abs(cost_s - best) <= 1e-9 * max(1.0, best)
    # D_r A D_c is an I-matrix: |entries| <= 1, = 1 on the matched ones
    rows = np.repeat(np.arange(n), np.diff(sp.rowptr))
    s = np.abs(info["row_scale"][rows] * sp.vals * info["col_scale"][sp.colidx])
    assert s.max() <= 1.0 + 1e-12
    matched = sigma[rows] == sp.colidx
    assert np.allclose(s[matched], 1.0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,k0,density,seed", [(500, 4, 0.5, 1), (3000, 10, 0.3, 2),
                                               (4000, 25, 0.15, 3)])
def test_cuthill_mckee_and_drop_equal_the_oracle(n, k0, density, seed):
    """The same ordering as the oracle's Cuthill-McKee on the boosted
    structure (deterministic tie-breaks), the same half-bandwidth, and the
    same drop-off K for several fractions."""
    sp = sapgen.make_sparse_problem(n, k0, density=density, seed=seed)
    sigma = osp.db_matching(n, sp.rowptr, sp.colidx, sp.vals)[0].astype(np.int64)
    B = osp.permute_csr(n, sp.rowptr, sp.colidx, sp.vals, sigma, np.arange(n))
    order, kk = osp.cuthill_mckee(n, B.indptr, B.indices)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    full = plan(sp).info()
    assert np.array_equal(full["new_col"], pos)
    assert np.array_equal(full["new_row"], pos[sigma])
    assert full["k_full"] == kk
    Ah = osp.permute_csr(n, sp.rowptr, sp.colidx, sp.vals, full["new_row"], full["new_col"],
                         full["row_scale"], full["col_scale"])
    assert osp.half_bandwidth(n, Ah.indptr, Ah.indices, np.arange(n)) == kk
    for frac in (1e-3, 2e-2):
        assert plan(sp, drop=frac).info()["k"] == osp.drop_k(n, Ah.indptr, Ah.indices, Ah.data, frac)
    assert kk <= 3 * k0                     # the hidden band is recovered


def test_analysis_stage_times():
    """sap_sparse_times: three non-negative host times, whose sum is within
    the wall time of sap_sparse_create; without reordering the matching and
    Cuthill-McKee stages do nothing measurable next to the full analysis."""
    import time
    sp = sapgen.make_sparse_problem(20000, 10, density=0.3, seed=15)
    t0 = time.perf_counter()
    pl = plan(sp)
    wall = (time.perf_counter() - t0) * 1e3
    t = pl.times()
    assert set(t) == {"t_db_ms", "t_cm_ms", "t_drop_ms"}
    assert all(v >= 0.0 for v in t.values())
    assert sum(t.values()) <= wall * 1.05 + 1.0
    assert t["t_db_ms"] > 0.0 and t["t_cm_ms"] > 0.0
    t_id = plan(sp, db=False, cm=False).times()
    assert t_id["t_db_ms"] + t_id["t_cm_ms"] < t["t_db_ms"] + t["t_cm_ms"]


def test_without_reordering_is_the_identity():
    sp = sapgen.make_sparse_problem(800, 5, seed=4)
    info = plan(sp, db=False, cm=False).info()
    assert np.array_equal(info["new_row"], np.arange(800))
    assert np.array_equal(info["new_col"], np.arange(800))
    assert np.all(info["row_scale"] == 1.0) and np.all(info["col_scale"] == 1.0)


def test_structurally_singular_is_reported(lib):
    from paper_1509_07919_amd import SapError, sap
    # rows 0 and 1 both only in column 0
    rowptr = np.array([0, 1, 2, 4], dtype=np.int64)
    colidx = np.array([0, 0, 1, 2], dtype=np.int32)
    vals = np.array([1.0, 2.0, 3.0, 4.0])
    from paper_1509_07919_amd import SapSparse
    with pytest.raises(SapError) as e:
        SapSparse(3, rowptr, colidx, vals)
    assert e.value.code == sap.SAP_ERR_SINGULAR


@pytest.mark.parametrize("n,k0,density,seed", [(300, 3, 0.6, 21), (2000, 8, 0.3, 22)])
def test_oracle_duals_are_feasible_and_tight(n, k0, density, seed):
    """Reduced costs c_ij - u_i - v_j >= 0 on every edge and 0 on the
    matched ones (LP duality: the matching is then optimal), so
    exp(u_i)/a_i |a_ij| exp(v_j) <= 1 with equality on the matching."""
    sp = sapgen.make_sparse_problem(n, k0, density=density, seed=seed)
    sigma, cost, u, v = osp.db_matching_duals(n, sp.rowptr, sp.colidx, sp.vals)
    C = osp.db_costs(n, sp.rowptr, sp.colidx, sp.vals).tocoo()
    red = C.data - u[C.row] - v[C.col]
    assert red.min() >= -1e-12
    assert np.abs(red[sigma[C.row] == C.col]).max() <= 1e-12
    assert abs(u.sum() + v.sum() - cost) <= 1e-9 * max(1.0, cost)


def test_invalid_csr_is_refused():
    """A repeated (row, column), a non-finite value, a column out of range and
    a decreasing rowptr are refused with SAP_ERR_INVALID."""
    from paper_1509_07919_amd import SapError, SapSparse, sap
    good = (np.array([0, 2, 4], dtype=np.int64), np.array([0, 1, 0, 1], dtype=np.int32),
            np.array([4.0, 1.0, 1.0, 4.0]))
    SapSparse(2, *good).close()
    bad = [
        (good[0], np.array([0, 0, 0, 1], dtype=np.int32), good[2]),          # repeated column
        (good[0], good[1], np.array([4.0, np.nan, 1.0, 4.0])),               # NaN
        (good[0], good[1], np.array([4.0, 1.0, np.inf, 4.0])),               # inf
        (good[0], np.array([0, 2, 0, 1], dtype=np.int32), good[2]),          # out of range
        (np.array([0, 3, 2], dtype=np.int64), good[1][:2], good[2][:2]),     # decreasing rowptr
    ]
    for rp, ci, va in bad:
        with pytest.raises(SapError) as e:
            SapSparse(2, rp, ci, va)
        assert e.value.code == sap.SAP_ERR_INVALID


def _csr_from_dense(A):
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
    return n, rowptr, cols.astype(np.int32), A[rows, cols].astype(np.float64)


def _check_against_oracle(A):
    from paper_1509_07919_amd import SapSparse
    n, rowptr, colidx, vals = _csr_from_dense(A)
    sigma_o, cost_o = osp.db_matching(n, rowptr, colidx, vals)
    info = SapSparse(n, rowptr, colidx, vals, db=True, cm=False).info()
    sigma = info["new_row"].astype(np.int64)
    assert abs(osp.matching_cost(n, rowptr, colidx, vals, sigma) - cost_o) <= 1e-12 * max(1.0, cost_o)
    s = np.abs(info["row_scale"][:, None] * A * info["col_scale"][None, :])
    assert s.max() <= 1.0 + 1e-12
    assert np.allclose(s[np.arange(n), sigma], 1.0, rtol=1e-12, atol=0)
    return sigma, sigma_o


def test_matching_edge_cases():
    """N = 1; a permutation matrix (the only perfect matching); a cyclic
    structure whose heaviest entries all sit in one column, so the initial
    greedy match leaves rows for long augmenting paths; a block of equal
    entries (many optimal matchings: costs and scaling compared, not the
    permutation)."""
    sigma, _ = _check_against_oracle(np.array([[3.0]]))
    assert list(sigma) == [0]
    P = np.zeros((6, 6))
    perm = [3, 0, 5, 1, 4, 2]
    P[np.arange(6), perm] = [2.0, -1.0, 0.5, 4.0, -3.0, 1.0]
    sigma, sigma_o = _check_against_oracle(P)
    assert list(sigma) == perm and list(sigma_o) == perm
    n = 9
    C = np.zeros((n, n))
    for i in range(n):
        C[i, 0] = 10.0 + i          # every row's heaviest entry in column 0
        C[i, (i + 1) % n] = 1.0 + 0.1 * i
        C[i, i] = 0.5 + 0.01 * i
    sigma, sigma_o = _check_against_oracle(C)
    assert np.array_equal(sigma, sigma_o)
    E = np.ones((5, 5))
    _check_against_oracle(E)


def test_cuthill_mckee_disconnected_and_diagonal():
    """A diagonal matrix (half-bandwidth 0, identity order) and a structure of
    three disconnected paths: the library's order equals the oracle's."""
    from paper_1509_07919_amd import SapSparse
    n, rowptr, colidx, vals = _csr_from_dense(np.diag(np.arange(1.0, 8.0)))
    info = SapSparse(n, rowptr, colidx, vals, db=False, cm=True).info()
    assert info["k_full"] == 0 and info["k"] == 0
    A = np.eye(12) * 4.0
    for a, b in ((0, 7), (7, 3), (3, 10), (1, 5), (5, 11), (2, 9), (9, 4), (4, 6), (6, 8)):
        A[a, b] = A[b, a] = 1.0
    n, rowptr, colidx, vals = _csr_from_dense(A)
    info = SapSparse(n, rowptr, colidx, vals, db=False, cm=True).info()
    order, kk = osp.cuthill_mckee(n, rowptr, colidx)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    assert np.array_equal(info["new_col"], pos)
    assert info["k_full"] == kk == 1
