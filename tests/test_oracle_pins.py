"""Pins for the CPU oracle against things other than itself: the paper's
storage example, exact rational arithmetic, LAPACK/SciPy library routines,
closed forms and exact special cases of the SaP method."""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sps
import scipy.sparse.linalg as spla

import sapgen
import oracle
from oracle import (DirectLU, SapPrecond, bandmv, band_get, bicgstab_l,
                    gradients, partition, solve_direct, _load, _p)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(pb):
    return sapgen.band_to_dense(pb.band, pb.n, pb.k)


# ------------------------------------------------------------------ layout

def test_band_layout_matches_paper_example():
    """Sec. 3.1 storage example, N=8, K=2: every printed position a_{r,c} is
    where our layout puts it, and '*' slots are exactly the padding."""
    n, k = 8, 2
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "band_layout_n8k2.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == n and all(len(r) == 2 * k + 1 for r in rows)
    a = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            if abs(r - c) <= k:
                a[r, c] = 10 * (r + 1) + (c + 1)
    band = sapgen.dense_to_band(a, k, pad=np.nan)
    for c, row in enumerate(rows):              # storage row c = matrix column c
        for q, tok in enumerate(row):
            v = band[q * n + c]                 # column-major: column q contiguous
            if tok == "*":
                assert np.isnan(v)
            else:
                rr, cc = (int(t) for t in tok.split(","))
                assert cc - 1 == c
                assert v == 10 * rr + cc
                assert sapgen.band_index(n, k, rr - 1, cc - 1) == q * n + c
                assert band_get(band, n, k, rr - 1, cc - 1) == v


def test_partition_rule():
    """Sec. 3.1: first P_r blocks get floor(N/P)+1 rows, N = P*floor(N/P)+P_r."""
    sizes, starts = partition(500_000, 128)
    assert (sizes[:32] == 3907).all() and (sizes[32:] == 3906).all()
    assert sizes.sum() == 500_000 and starts[0] == 0
    assert (np.diff(starts) == sizes[:-1]).all()
    assert list(partition(10, 3)[0]) == [4, 3, 3]
    assert list(partition(200_000, 64)[0]) == [3125] * 64
    assert list(partition(7, 7)[0]) == [1] * 7
    with pytest.raises(ValueError):
        partition(5, 6)


def test_generator_dominance_and_rhs():
    """The generated rows have |a_ii| = d * sum|a_ij| (eq:diagDominanceDef
    with equality); b = A x_true."""
    for d, scale in [(1.0, 0.0), (0.5, 0.0), (0.1, 2.0)]:
        pb = sapgen.make_problem(300, 9, d=d, seed=4, row_scale_decades=scale)
        a = dense(pb)
        off = np.abs(a).sum(1) - np.abs(np.diag(a))
        np.testing.assert_allclose(np.abs(np.diag(a)), d * off, rtol=1e-14)
        np.testing.assert_allclose(a @ pb.x_true, pb.b, rtol=1e-12, atol=1e-12)


# -------------------------------------------------------------------- SpMV

@pytest.mark.parametrize("n,k", [(1, 0), (5, 4), (37, 6), (300, 11)])
def test_bandmv_matches_dense(n, k):
    pb = sapgen.make_problem(n, k, seed=11, pad=np.nan)
    a = np.nan_to_num(dense(pb))
    v = sapgen.splitmix64_uniform(1, 9, np.arange(n))
    np.testing.assert_allclose(bandmv(pb.band, n, k, v), a @ v, rtol=0, atol=1e-13)
    np.testing.assert_allclose(bandmv(pb.band, n, k, v, trans=True), a.T @ v,
                               rtol=0, atol=1e-13)


# ------------------------------------------------------------ direct solve

def _exact_solve(a, b):
    """Gaussian elimination in exact rational arithmetic (floats are dyadic
    rationals, so the inputs are represented exactly)."""
    n = len(b)
    m = [[Fraction(float(a[i, j])) for j in range(n)] + [Fraction(float(b[i]))]
         for i in range(n)]
    for j in range(n):
        p = next(i for i in range(j, n) if m[i][j] != 0)
        m[j], m[p] = m[p], m[j]
        for i in range(j + 1, n):
            f = m[i][j] / m[j][j]
            for c in range(j, n + 1):
                m[i][c] -= f * m[j][c]
    x = [Fraction(0)] * n
    for j in range(n - 1, -1, -1):
        s = m[j][n] - sum(m[j][c] * x[c] for c in range(j + 1, n))
        x[j] = s / m[j][j]
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("n,k,d", [(9, 2, 1.0), (12, 3, 0.3), (10, 9, 0.05)])
def test_direct_solve_vs_exact_rational(n, k, d):
    pb = sapgen.make_problem(n, k, d=d, seed=5)
    a = dense(pb)
    xe = _exact_solve(a, pb.b)
    xte = _exact_solve(a.T, pb.b)
    cond = np.linalg.cond(a)
    tol = 1e-15 * cond * 20
    np.testing.assert_allclose(solve_direct(pb.band, n, k, pb.b), xe, rtol=0,
                               atol=tol * np.abs(xe).max())
    np.testing.assert_allclose(solve_direct(pb.band, n, k, pb.b, trans=True), xte,
                               rtol=0, atol=tol * np.abs(xte).max())


@pytest.mark.parametrize("n,k,d", [(64, 5, 1.0), (64, 20, 0.1), (500, 30, 0.5)])
def test_direct_solve_vs_lapack(n, k, d):
    """O2 against LAPACK gesv (dense) and gbsv (scipy.solve_banded)."""
    pb = sapgen.make_problem(n, k, d=d, seed=6)
    a = dense(pb)
    lu = DirectLU(pb.band, n, k)
    x = lu.solve(pb.b)
    xt = lu.solve(pb.b, trans=True)
    cond = np.linalg.cond(a, 1)
    tol = 1e-15 * cond * 10
    np.testing.assert_allclose(x, np.linalg.solve(a, pb.b), rtol=0, atol=tol)
    np.testing.assert_allclose(xt, np.linalg.solve(a.T, pb.b), rtol=0, atol=tol)
    ab = np.zeros((2 * k + 1, n))             # LAPACK band storage
    for q in range(2 * k + 1):                 # ab[k + i - j, j] = a[i, j]
        ab[q] = pb.band2d()[q]
    np.testing.assert_allclose(x, sla.solve_banded((k, k), ab, pb.b), rtol=0, atol=tol)
    assert np.linalg.norm(a @ x - pb.b) / np.linalg.norm(pb.b) <= 1e-13
    est = lu.cond1_estimate(pb.band)
    assert cond / 3 <= est <= cond * (1 + 1e-8)


def test_direct_solve_residual_large():
    n, k = 20_000, 10
    pb = sapgen.make_problem(n, k, seed=7)
    x = solve_direct(pb.band, n, k, pb.b)
    r = pb.b - bandmv(pb.band, n, k, x)
    assert np.linalg.norm(r) / np.linalg.norm(pb.b) <= 1e-12
    np.testing.assert_allclose(x, pb.x_true, rtol=0, atol=1e-10)


# ---------------------------------------------------- block LU / UL / boost

def _block_window(pb, s0, nb):
    f = np.empty(nb * (2 * pb.k + 1))
    _load().orc_block_load(pb.n, pb.k, _p(pb.band), s0, nb, _p(f))
    return f


def _window_to_dense(f, nb, k):
    m = np.zeros((nb, nb))
    for r in range(nb):
        for c in range(max(0, r - k), min(nb, r + k + 1)):
            m[r, c] = f[r * (2 * k + 1) + c - r + k]
    return m


def test_block_lu_ul_reconstruct():
    """L U = A_i and U' L' = A_i (no pivoting); UL(A) = J LU(J A J) J."""
    import ctypes
    pb = sapgen.make_problem(120, 6, d=1.0, seed=8)
    s0, nb, k = 30, 50, pb.k
    a = dense(pb)[s0:s0 + nb, s0:s0 + nb]
    nbst = ctypes.c_int32(0)
    f = _block_window(pb, s0, nb)
    assert _load().orc_block_lu(nb, k, _p(f), -1.0, ctypes.byref(nbst)) == 0
    m = _window_to_dense(f, nb, k)
    L, U = np.tril(m, -1) + np.eye(nb), np.triu(m)
    np.testing.assert_allclose(L @ U, a, atol=1e-13 * np.abs(a).max())
    g = _block_window(pb, s0, nb)
    assert _load().orc_block_ul(nb, k, _p(g), -1.0, ctypes.byref(nbst)) == 0
    m2 = _window_to_dense(g, nb, k)
    Up, Lp = np.triu(m2, 1) + np.eye(nb), np.tril(m2)
    np.testing.assert_allclose(Up @ Lp, a, atol=1e-13 * np.abs(a).max())
    # J LU(J A J) J: reversed problem through the LU routine
    J = np.eye(nb)[::-1]
    h = sapgen.dense_to_band(J @ a @ J, k)
    hw = np.empty(nb * (2 * k + 1))
    _load().orc_block_load(nb, k, _p(h), 0, nb, _p(hw))
    _load().orc_block_lu(nb, k, _p(hw), -1.0, ctypes.byref(nbst))
    m3 = _window_to_dense(hw, nb, k)
    np.testing.assert_allclose(J @ (np.tril(m3, -1) + np.eye(nb)) @ J, Up, atol=1e-12)
    np.testing.assert_allclose(J @ np.triu(m3) @ J, Lp, atol=1e-12)


def test_block_lu_matches_scipy_without_pivoting():
    """On a strictly diagonally dominant block, partial pivoting never swaps,
    so LAPACK getrf's L and U equal the no-pivot factors."""
    import ctypes
    pb = sapgen.make_problem(60, 4, d=2.0, seed=9)
    k, nb = pb.k, 60
    f = _block_window(pb, 0, nb)
    nbst = ctypes.c_int32(0)
    _load().orc_block_lu(nb, k, _p(f), -1.0, ctypes.byref(nbst))
    P, L, U = sla.lu(dense(pb))
    assert np.array_equal(P, np.eye(nb))
    m = _window_to_dense(f, nb, k)
    np.testing.assert_allclose(np.tril(m, -1), np.tril(L, -1), atol=1e-14)
    np.testing.assert_allclose(np.triu(m), U, atol=1e-13)


def test_pivot_boost_exact_perturbation():
    """Sec. 2.2: a pivot below tau is replaced by +-tau; the factors are those
    of A + delta A with delta A on that one diagonal entry."""
    import ctypes
    n, k = 12, 2
    pb = sapgen.make_problem(n, k, seed=10)
    a = dense(pb)
    a[0, 0] = 0.0                               # first pivot exactly zero
    band = sapgen.dense_to_band(a, k)
    f = np.empty(n * (2 * k + 1))
    _load().orc_block_load(n, k, _p(band), 0, n, _p(f))
    nbst = ctypes.c_int32(0)
    tau = 1e-3
    assert _load().orc_block_lu(n, k, _p(f), tau, ctypes.byref(nbst)) == 0
    assert nbst.value == 1
    m = _window_to_dense(f, n, k)
    L, U = np.tril(m, -1) + np.eye(n), np.triu(m)
    ap = a.copy()
    ap[0, 0] = tau                              # sign of 0 taken as +
    np.testing.assert_allclose(L @ U, ap, atol=1e-12)
    g = np.empty(n * (2 * k + 1))
    _load().orc_block_load(n, k, _p(band), 0, n, _p(g))
    assert _load().orc_block_lu(n, k, _p(g), -1.0, ctypes.byref(nbst)) == 1  # disabled


# ------------------------------------------------------------- spike tips

@pytest.mark.parametrize("d", [1.0, 0.3])
def test_tips_equal_dense_spike_tips(d):
    """eq:LeftRightSpikes: V_i = A_i^{-1}[0;0;B_i], W_i = A_i^{-1}[C_i;0;0];
    the corner formulas must give their bottom/top K rows."""
    n, k, p = 160, 5, 4
    pb = sapgen.make_problem(n, k, d=d, seed=12)
    a = dense(pb)
    M = SapPrecond(pb.band, n, k, p, coupled=True, boost_eps=-1.0)
    for i in range(p - 1):
        s0, nb = int(M.starts[i]), int(M.sizes[i])
        s1, nb1 = int(M.starts[i + 1]), int(M.sizes[i + 1])
        Ai = a[s0:s0 + nb, s0:s0 + nb]
        Aj = a[s1:s1 + nb1, s1:s1 + nb1]
        B = a[s1 - k:s1, s1:s1 + k]
        C = a[s1:s1 + k, s1 - k:s1]
        np.testing.assert_array_equal(M.B[i], B)
        np.testing.assert_array_equal(M.C[i], C)
        assert np.allclose(np.triu(B, 1), 0) and np.allclose(np.tril(C, -1), 0)
        rhs = np.zeros((nb, k)); rhs[-k:] = B
        Vfull = np.linalg.solve(Ai, rhs)
        rhs = np.zeros((nb1, k)); rhs[:k] = C
        Wfull = np.linalg.solve(Aj, rhs)
        np.testing.assert_allclose(M.V[i], Vfull[-k:], atol=1e-12)
        np.testing.assert_allclose(M.W[i], Wfull[:k], atol=1e-12)


def _brute_force_truncated(a, n, k, sizes, starts, r):
    """SaP-C from the dense formulas: g = D^{-1} r, full spikes by dense
    solves, each 2K x 2K R_i [x_i^(b); x_{i+1}^(t)] = [g_i^(b); g_{i+1}^(t)]
    with R_i = [[I, V_i^(b)], [W_{i+1}^(t), I]] (N_i = M_i = 0), then the
    purification solves."""
    p = len(sizes)
    blocks = [a[s:s + m, s:s + m] for s, m in zip(starts, sizes)]
    g = np.concatenate([np.linalg.solve(B_, r[s:s + m])
                        for B_, s, m in zip(blocks, starts, sizes)])
    rp = r.copy()
    for i in range(p - 1):
        s1 = starts[i + 1]
        B = a[s1 - k:s1, s1:s1 + k]
        C = a[s1:s1 + k, s1 - k:s1]
        rhs = np.zeros((sizes[i], k)); rhs[-k:] = B
        Vb = np.linalg.solve(blocks[i], rhs)[-k:]
        rhs = np.zeros((sizes[i + 1], k)); rhs[:k] = C
        Wt = np.linalg.solve(blocks[i + 1], rhs)[:k]
        R = np.block([[np.eye(k), Vb], [Wt, np.eye(k)]])
        xh = np.linalg.solve(R, np.concatenate([g[s1 - k:s1], g[s1:s1 + k]]))
        xb, xt = xh[:k], xh[k:]
        rp[s1 - k:s1] -= B @ xt
        rp[s1:s1 + k] -= C @ xb
    return np.concatenate([np.linalg.solve(B_, rp[s:s + m])
                           for B_, s, m in zip(blocks, starts, sizes)])


@pytest.mark.parametrize("n,k,p,d", [(90, 4, 3, 1.0), (203, 6, 5, 0.4), (64, 8, 4, 1.0)])
def test_sapc_apply_equals_truncated_reduced_system(n, k, p, d):
    pb = sapgen.make_problem(n, k, d=d, seed=13)
    a = dense(pb)
    M = SapPrecond(pb.band, n, k, p, coupled=True, boost_eps=-1.0)
    r = sapgen.splitmix64_uniform(2, 7, np.arange(n))
    want = _brute_force_truncated(a, n, k, list(M.sizes), list(M.starts), r)
    np.testing.assert_allclose(M.apply(r), want, atol=1e-11 * np.abs(want).max())


def test_sapd_apply_equals_block_solves():
    n, k, p = 101, 7, 6
    pb = sapgen.make_problem(n, k, seed=14)
    a = dense(pb)
    M = SapPrecond(pb.band, n, k, p, coupled=False, boost_eps=-1.0)
    r = sapgen.splitmix64_uniform(3, 7, np.arange(n))
    want = np.concatenate([np.linalg.solve(a[s:s + m, s:s + m], r[s:s + m])
                           for s, m in zip(M.starts, M.sizes)])
    np.testing.assert_allclose(M.apply(r), want, atol=1e-12)


@pytest.mark.parametrize("p,coupled", [(1, False), (1, True), (2, True)])
def test_exact_special_cases(p, coupled):
    """P=1 (either mode) and SaP-C with P=2 drop nothing, so M^{-1} = A^{-1};
    BiCGStab(2) then exits at the first exit point, 0.25 iterations."""
    n, k = 120, 5
    pb = sapgen.make_problem(n, k, seed=15)
    a = dense(pb)
    M = SapPrecond(pb.band, n, k, p, coupled, boost_eps=-1.0)
    r = sapgen.splitmix64_uniform(4, 7, np.arange(n))
    np.testing.assert_allclose(M.apply(r), np.linalg.solve(a, r), atol=1e-12)
    np.testing.assert_allclose(M.apply_t(r), np.linalg.solve(a.T, r), atol=1e-12)
    res = bicgstab_l(lambda v: bandmv(pb.band, n, k, v), M.apply, pb.b, tol=1e-10)
    assert res.converged and res.iters == 0.25
    np.testing.assert_allclose(res.x, pb.x_true, atol=1e-12)


def test_block_diagonal_matrix_is_exact():
    """With B_i = C_i = 0 the truncation drops nothing: M^{-1} = A^{-1}."""
    n, k, p = 90, 3, 3
    pb = sapgen.make_problem(n, k, seed=16)
    a = dense(pb)
    for s in (30, 60):
        a[s - k:s, s:s + k] = 0.0
        a[s:s + k, s - k:s] = 0.0
    band = sapgen.dense_to_band(a, k)
    for coupled in (False, True):
        M = SapPrecond(band, n, k, p, coupled, boost_eps=-1.0)
        r = sapgen.splitmix64_uniform(5, 7, np.arange(n))
        np.testing.assert_allclose(M.apply(r), np.linalg.solve(a, r), atol=1e-12)


@pytest.mark.parametrize("coupled", [False, True])
def test_transpose_identity(coupled):
    """<M^{-1} u, v> = <u, M^{-T} v> and <A u, v> = <u, A^T v>."""
    n, k, p = 300, 7, 5
    pb = sapgen.make_problem(n, k, d=0.6, seed=17)
    M = SapPrecond(pb.band, n, k, p, coupled)
    u = sapgen.splitmix64_uniform(6, 7, np.arange(n))
    v = sapgen.splitmix64_uniform(7, 7, np.arange(n))
    lhs, rhs = M.apply(u) @ v, u @ M.apply_t(v)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(u) * np.linalg.norm(v))
    lhs, rhs = bandmv(pb.band, n, k, u) @ v, u @ bandmv(pb.band, n, k, v, trans=True)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------- Krylov

def test_bicgstab1_matches_scipy_bicgstab():
    """For l = 1, BiCGStab(l) is van der Vorst's BiCGStab: same iterates as
    SciPy's bicgstab after the same number of steps (no preconditioner)."""
    n = 80
    rng = np.random.default_rng(0)
    a = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    for m in (1, 2, 5):
        ours = bicgstab_l(lambda v: a @ v, lambda v: v, b, tol=1e-300, maxit=m, ell=1)
        theirs, _ = spla.bicgstab(sps.csr_matrix(a), b, rtol=1e-300, atol=0.0,
                                  maxiter=m)
        np.testing.assert_allclose(ours.x, theirs, rtol=1e-11, atol=1e-13)


def test_bicgstab2_minimal_polynomial_degree_two():
    """If the operator has a degree-2 minimal polynomial, two BiCG steps reach
    the exact solution: exit at the second exit point, 0.75 iterations."""
    n = 50
    rng = np.random.default_rng(1)
    uvec, vvec = rng.standard_normal(n), rng.standard_normal(n)
    a = 2.0 * np.eye(n) + np.outer(uvec, vvec) / n     # I-scaled + rank one
    b = rng.standard_normal(n)
    res = bicgstab_l(lambda v: a @ v, lambda v: v, b, tol=1e-12, ell=2)
    assert res.converged and res.iters == 0.75
    np.testing.assert_allclose(res.x, np.linalg.solve(a, b), atol=1e-12)


def _similar_to_diag(n, eigs, seed):
    """A = S diag(lam) S^{-1}, nonsymmetric, whose minimal polynomial has
    degree len(set(eigs)) (each eigenvalue repeated)."""
    rng = np.random.default_rng(seed)
    lam = np.array([eigs[i % len(eigs)] for i in range(n)], dtype=np.float64)
    S = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    return S @ np.diag(lam) @ np.linalg.inv(S), rng.standard_normal(n)


@pytest.mark.parametrize("eigs,exit_iters", [((1.0, 2.0, 4.0), 1.25),
                                             ((1.0, 2.0, 3.0, 5.0), 1.75)])
def test_bicgstab2_finite_termination_through_the_mr_part(eigs, exit_iters):
    """BiCGStab(2) multiplies the BiCG residual polynomial by its MR
    polynomial, so once the BiCG steps reach the degree d of the minimal
    polynomial the residual is zero.  For d = 3 that is the first BiCG step
    of the second iteration (1.25 iterations), for d = 4 the second (1.75):
    both come after a minimal-residual part, whose updates of u_0 (gamma),
    x (gamma_1, gamma''_1) and r_0 (gamma') must all be right for the third
    and fourth BiCG steps to stay exact (Sleijpen-Fokkema 1993)."""
    n = 40
    a, b = _similar_to_diag(n, eigs, seed=11)
    res = bicgstab_l(lambda v: a @ v, lambda v: v, b, tol=1e-11, ell=2)
    assert res.converged and res.restarts == 0 and res.iters == exit_iters
    np.testing.assert_allclose(res.x, np.linalg.solve(a, b), rtol=0,
                               atol=1e-10 * np.abs(np.linalg.solve(a, b)).max())


@pytest.mark.parametrize("precond", [False, True])
def test_bicgstab2_recursion_invariant_and_mr_orthogonality(precond):
    """Two properties of every BiCGStab(2) iterate, checked on a small
    nonsymmetric system (with and without a left preconditioner):
    * at every exit point the recursive residual equals the true one,
      r_0 = M^{-1}(b - A x) (the x updates by alpha, gamma_1, gamma''_1 are
      consistent with the r_0 updates);
    * after each minimal-residual part, r_0 is orthogonal to the
      Gram-Schmidt-orthogonalized r_1 and r_2: the MR coefficients gamma'
      minimize ||r_0 - gamma'_1 r_1 - gamma'_2 r_2||."""
    n = 60
    rng = np.random.default_rng(3)
    a = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    a[0, :] *= 0.2                                   # spread the spectrum
    b = rng.standard_normal(n)
    minv = (np.linalg.inv(np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n))
            if precond else np.eye(n))
    seen = {"bicg": 0, "mr": 0}

    def observe(kind, napply, x, r, u):
        seen[kind] += 1
        t = minv @ (b - a @ x)
        assert np.linalg.norm(r[0] - t) <= 1e-12 * np.linalg.norm(minv @ b)
        if kind == "mr":
            for j in (1, 2):
                c = abs(r[0] @ r[j]) / (np.linalg.norm(r[0]) * np.linalg.norm(r[j]))
                assert c <= 1e-12
            c12 = abs(r[1] @ r[2]) / (np.linalg.norm(r[1]) * np.linalg.norm(r[2]))
            assert c12 <= 1e-12

    res = bicgstab_l(lambda v: a @ v, lambda v: minv @ v, b, tol=1e-300, maxit=4,
                     ell=2, observe=observe)
    assert seen["mr"] == 4 and seen["bicg"] == 8 and res.restarts == 0


def test_bicgstab2_scalar_operator_first_exit():
    n = 30
    b = np.arange(1.0, n + 1)
    res = bicgstab_l(lambda v: 3.0 * v, lambda v: v, b, tol=1e-12)
    assert res.converged and res.iters == 0.25
    np.testing.assert_allclose(res.x, b / 3.0, rtol=1e-15)


def test_reliable_updates_with_a_low_precision_preconditioner():
    """The inverse of a nearby matrix (relative distance ~1e-6), its output
    rounded to FP32: the recursive residual falls far below the true one,
    which stalls near 1e-7.  The reliable-update rule restarts as soon as the
    recursive residual has dropped by 1e-4 and reaches 1e-12 in fewer operator
    applications than restarting only at the threshold; both end at the exact
    solution."""
    n = 60
    rng = np.random.default_rng(2)
    a = np.eye(n) * 5 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    ainv = np.linalg.inv(a + 1e-6 * rng.standard_normal((n, n)))
    pre = lambda v: (ainv @ v).astype(np.float32).astype(np.float64)
    plain = bicgstab_l(lambda v: a @ v, pre, b, tol=1e-12)
    rel = bicgstab_l(lambda v: a @ v, pre, b, tol=1e-12, reliable=1e-4)
    xs = np.linalg.solve(a, b)
    for res in (plain, rel):
        assert res.converged and res.rel_resid_true <= 1e-12
        np.testing.assert_allclose(res.x, xs, rtol=0, atol=1e-10 * np.abs(xs).max())
    assert rel.restarts >= 1 and rel.iters < plain.iters
    off = bicgstab_l(lambda v: a @ v, pre, b, tol=1e-12, reliable=0.0)
    assert np.array_equal(off.x, plain.x) and off.iters == plain.iters


@pytest.mark.parametrize("coupled,p,d", [(False, 16, 1.0), (True, 8, 1.0), (True, 8, 0.5)])
def test_sap_bicgstab2_converges_to_direct(coupled, p, d):
    from oracle import sap_solve
    n, k = 4000, 10
    pb = sapgen.make_problem(n, k, d=d, seed=18)
    x, res, M = sap_solve(pb.band, n, k, pb.b, p, coupled, tol=1e-12)
    assert res.converged and res.rel_resid_true <= 1e-12
    xd = solve_direct(pb.band, n, k, pb.b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-9
    assert res.iters == int(res.iters * 4) / 4                # quarters


def test_coupled_needs_fewer_iterations_than_decoupled():
    """Sec. 4.1.1: the coupled preconditioner is of better quality."""
    from oracle import sap_solve
    n, k, p = 20_000, 20, 16
    pb = sapgen.make_problem(n, k, d=1.0, seed=19)
    _, rd, _ = sap_solve(pb.band, n, k, pb.b, p, False, tol=1e-10)
    _, rc, _ = sap_solve(pb.band, n, k, pb.b, p, True, tol=1e-10)
    assert rc.converged and rd.converged and rc.iters < rd.iters


# ------------------------------------------------------------- gradients

def test_gradients_central_differences():
    """L = 0.5||x - x_t||^2, x = A^{-1} b.  dL/db is exact for this quadratic
    (central differences exact up to rounding); dL/dA band by FD with h=1e-6."""
    n, k = 40, 3
    pb = sapgen.make_problem(n, k, seed=20)
    xt = sapgen.normal_draws(20, sapgen.STREAM_XTARGET, n)
    x, gb, ga = gradients(pb.band, n, k, pb.b, xt)

    def loss(band, b):
        y = solve_direct(band, n, k, b)
        return 0.5 * np.sum((y - xt) ** 2)

    h = 1e-6
    for j in (0, 7, 39):
        e = np.zeros(n); e[j] = h
        fd = (loss(pb.band, pb.b + e) - loss(pb.band, pb.b - e)) / (2 * h)
        assert abs(fd - gb[j]) <= 1e-7 * max(1.0, abs(gb[j]))
    for (r, c) in [(0, 0), (5, 3), (10, 13), (39, 36)]:
        pos = (k + r - c) * n + c
        bp, bm = pb.band.copy(), pb.band.copy()
        bp[pos] += h; bm[pos] -= h
        fd = (loss(bp, pb.b) - loss(bm, pb.b)) / (2 * h)
        assert abs(fd - ga[pos]) <= 1e-6 * max(1.0, abs(ga[pos]))
    # padding slots of the gradient are zero
    assert ga[(k - 1) * n + 0] == 0.0


def _float32_dinv(band, n, k, p, r):
    """An independent FP32 evaluation of D^{-1} r: each block densely in
    float32, LU without pivoting (no boost needed for these matrices), then
    the forward and backward substitutions, all in float32."""
    sizes, starts = oracle.partition(n, p)
    out = np.zeros(n)
    for nb, s0 in zip(sizes, starts):
        nb, s0 = int(nb), int(s0)
        A = np.array([[oracle.band_get(band, n, k, s0 + a, s0 + b) for b in range(nb)]
                      for a in range(nb)], dtype=np.float32)
        for j in range(nb):
            A[j + 1:j + k + 1, j] /= A[j, j]
            A[j + 1:j + k + 1, j + 1:j + k + 1] -= np.outer(A[j + 1:j + k + 1, j],
                                                           A[j, j + 1:j + k + 1])
        y = r[s0:s0 + nb].astype(np.float32)
        for j in range(nb):
            y[j + 1:j + k + 1] -= A[j + 1:j + k + 1, j] * y[j]
        for j in range(nb - 1, -1, -1):
            y[j] = y[j] / A[j, j]
            y[max(0, j - k):j] -= A[max(0, j - k):j, j] * y[j]
        out[s0:s0 + nb] = y
    return out


@pytest.mark.parametrize("d", [0.5, 0.12])
def test_fp32_error_model_against_float32_evaluation(d):
    """The FP32 error model of D^{-1} (first-order bound and its statistical
    version) against an actual float32 evaluation: every entry within the
    rigorous bound, and within 6 sigma of the statistical model, which is
    itself at most the bound."""
    n, k, p = 3200, 16, 4
    pb = sapgen.make_problem(n, k, d=d, seed=47)
    M = oracle.SapPrecond(pb.band, n, k, p, False, boost_eps=2.0 ** -23)
    r = sapgen.splitmix64_uniform(8, 7, np.arange(n))
    g = M.dinv(r)
    err = np.abs(_float32_dinv(pb.band, n, k, p, r) - g)
    bound = oracle.dinv_error_bound(M, r)
    sig = oracle.dinv_error_sigma(M, r)
    u = 2.0 ** -24
    assert np.all(err <= bound)
    assert np.all(err <= 6 * sig + 8 * u * np.abs(g))
    assert np.all(sig <= bound)
    # the errors are real: the model is not trivially loose everywhere
    assert (err / sig).max() >= 0.3


def test_fp32_error_model_of_a_diagonal_matrix():
    """K = 0: g = r / a, rounded twice (r and a to FP32) and once more by the
    division: |g_hat - g| <= 3u|g| + O(u^2), inside the bound."""
    n = 500
    pb = sapgen.make_problem(n, 0, d=1.0, seed=49)
    band = pb.band * (1.0 + sapgen.splitmix64_uniform(49, 6, np.arange(n)))
    M = oracle.SapPrecond(band, n, 0, 5, False, boost_eps=2.0 ** -23)
    r = sapgen.splitmix64_uniform(50, 7, np.arange(n))
    g = r / band
    bound = oracle.dinv_error_bound(M, r)
    u = 2.0 ** -24
    assert np.all(bound >= 3 * u * np.abs(g))
    assert np.all(bound <= 20 * u * np.abs(g))
    g32 = (r.astype(np.float32) / band.astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(g32 - g) <= bound)


# ------------------------------------------------ conjugate gradient (SPD)

def test_cg_iterates_match_scipy_cg():
    """The oracle's preconditioned CG (Saad Alg. 9.1) produces the same
    iterates as SciPy's cg with the same preconditioner, step by step."""
    n, k, p = 2000, 6, 5
    pb = sapgen.make_problem(n, k, d=1.02, seed=51, symmetric=True)
    M = SapPrecond(pb.band, n, k, p, False)
    A = sps.csr_matrix(sapgen.band_to_dense(pb.band, n, k))
    mine = []
    oracle.cg(lambda v: bandmv(pb.band, n, k, v), M.apply, pb.b, tol=1e-14, maxit=6,
              observe=lambda it, x, r: mine.append(x))
    ref = []
    Mop = spla.LinearOperator((n, n), matvec=M.apply)
    spla.cg(A, pb.b, M=Mop, rtol=0.0, atol=0.0, maxiter=6, callback=lambda xk: ref.append(xk.copy()))
    assert len(mine) == len(ref) == 6
    for a_, b_ in zip(mine, ref):
        assert np.abs(a_ - b_).max() <= 1e-12 * np.abs(b_).max()


def test_cg_finite_termination_three_eigenvalues():
    """CG on an SPD matrix with 3 distinct eigenvalues and no preconditioning
    reaches the solution in 3 steps (exact-arithmetic termination)."""
    n = 300
    diag = np.array([1.0, 4.0, 9.0])[np.arange(n) % 3]
    band = diag.copy()                       # K = 0 band layout: the diagonal
    xt = sapgen.splitmix64_uniform(52, 2, np.arange(n))
    b = diag * xt
    res = oracle.cg(lambda v: bandmv(band, n, 0, v), lambda v: v.copy(), b, tol=1e-13, maxit=10)
    assert res.converged and res.iters == 3.0 and res.restarts == 0
    assert np.abs(res.x - xt).max() <= 1e-13


def test_cg_exact_preconditioner_one_step():
    """P = 1: M = A (no boost), so z = A^{-1} r and the first CG step lands on
    the solution."""
    n, k = 1500, 9
    pb = sapgen.make_problem(n, k, d=1.1, seed=53, symmetric=True)
    x, res, _ = oracle.sap_solve_cg(pb.band, n, k, pb.b, 1, False, tol=1e-12)
    assert res.converged and res.iters == 1.0
    assert np.abs(x - pb.x_true).max() <= 1e-12


def test_cg_breakdown_on_indefinite_direction():
    """p^T A p = 0 for A = diag(1, -1) and b = (1, 1): CG breaks down."""
    band = np.array([1.0, -1.0])
    with pytest.raises(oracle.Breakdown):
        oracle.cg(lambda v: bandmv(band, 2, 0, v), lambda v: v.copy(), np.ones(2))


def test_spd_generator_is_symmetric_positive_definite():
    n, k = 400, 12
    pb = sapgen.make_problem(n, k, d=1.05, seed=54, symmetric=True)
    A = sapgen.band_to_dense(pb.band, n, k)
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0.0
    assert np.all(np.diag(A) > 0)
