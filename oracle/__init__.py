"""CPU oracle for the dense banded SaP solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package's ``smoke()`` check and the benchmark's
CPU-baseline leg may import this package.  It is plain, slow and sequential,
in float64, and shares no code with the GPU library (it neither imports it
nor is imported by it); the only module both sides use is ``sapgen``, which
draws the seeded inputs.

What it computes, and the passage each part follows (paper: Li, Serban,
Negrut, "Analysis of a splitting approach for the parallel solution of
linear systems on GPU cards", arXiv:1509.07919):

* ``solve_direct`` / ``DirectLU`` -- x = A^{-1} b and A^{-T} g by banded LU
  with partial pivoting.  This is the plain definition of the result the
  method reaches (the preconditioner changes the path, not the answer).
* ``partition`` -- block sizes, Sec. 3.1 "Number of partitions and partition
  size".
* ``SapPrecond`` -- the SaP preconditioner: block LU without pivoting with
  pivot boosting (Sec. 2.2 pivot-boosting paragraph), the UL factorization
  and the spike tips V_i^(b), W_{i+1}^(t) from the factor corners (Sec. 2.1,
  paragraph after the purification equations; eq:LeftRightSpikes), the
  truncated reduced systems and purification (eq:solveTopBottom and the
  purification equations that follow it), and the decoupled/coupled choice
  (Sec. 2.1.1).  ``apply_t`` is the exact transpose of ``apply``.
* ``bicgstab_l`` -- BiCGStab(l) of Sleijpen and Fokkema (ETNA 1, 1993; the
  paper's outer Krylov method, Sec. 2.1.1) with left preconditioning and the
  three exit points per l=2 iteration counted in quarters (Sec. 4.1.1).
* ``band_grad`` -- dL/dA restricted to the band, -lambda x^T.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sap_oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the C part with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        os.makedirs(_LIBDIR, exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, i32, dp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.orc_bandmv.argtypes = [i64, i32, dp, dp, dp, i32]
        lib.orc_gb_factor.argtypes = [i64, i32, dp, dp, dp]
        lib.orc_gb_factor.restype = i32
        lib.orc_gb_solve.argtypes = [i64, i32, dp, dp, dp, i32]
        lib.orc_block_load.argtypes = [i64, i32, dp, i64, i64, dp]
        lib.orc_block_maxabs.argtypes = [i64, i32, dp]
        lib.orc_block_maxabs.restype = ctypes.c_double
        lib.orc_block_lu.argtypes = [i64, i32, dp, ctypes.c_double,
                                     ctypes.POINTER(i32)]
        lib.orc_block_lu.restype = i32
        lib.orc_block_ul.argtypes = lib.orc_block_lu.argtypes
        lib.orc_block_ul.restype = i32
        lib.orc_block_solve.argtypes = [i64, i32, dp, dp, i32]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------- SpMV

def bandmv(band, n: int, k: int, v, trans: bool = False) -> np.ndarray:
    """y = A v (or A^T v) from the band layout, entry by entry."""
    band, v = _f64(band), _f64(v)
    y = np.empty(n, dtype=np.float64)
    _load().orc_bandmv(n, k, _p(band), _p(v), _p(y), int(bool(trans)))
    return y


def band_get(band, n: int, k: int, r: int, c: int) -> float:
    """a[r, c] from the band layout (0 outside the band)."""
    if abs(r - c) > k or not (0 <= r < n and 0 <= c < n):
        return 0.0
    return float(band[(k + r - c) * n + c])


# ------------------------------------------------------ direct solve (O2)

class DirectLU:
    """Banded LU with partial pivoting of the whole A; solves A x = b and
    A^T x = b.  The plain definition of x = A^{-1} b for parity checks."""

    def __init__(self, band, n: int, k: int):
        self.n, self.k = n, k
        self.lu = np.empty(n * (3 * k + 1), dtype=np.float64)
        self.ipiv = np.empty(n, dtype=np.int64)
        info = _load().orc_gb_factor(n, k, _p(_f64(band)), _p(self.lu),
                                     _p(self.ipiv))
        if info != 0:
            raise np.linalg.LinAlgError("exactly singular at column %d" % (info - 1))

    def solve(self, b, trans: bool = False) -> np.ndarray:
        x = np.array(b, dtype=np.float64, copy=True)
        _load().orc_gb_solve(self.n, self.k, _p(self.lu), _p(self.ipiv),
                             _p(x), int(bool(trans)))
        return x

    def cond1_estimate(self, band, iters: int = 5) -> float:
        """||A||_1 * est(||A^{-1}||_1), Hager's estimator (Higham's variant
        without the extra parallel test)."""
        n, k = self.n, self.k
        b2 = np.asarray(band).reshape(2 * k + 1, n)
        colsum = np.zeros(n)
        cols = np.arange(n)
        for q in range(2 * k + 1):
            d = q - k
            c = cols[max(0, -d):n - max(0, d)]
            colsum[c] += np.abs(b2[q, c])
        anorm = colsum.max()
        x = np.full(n, 1.0 / n)
        est = 0.0
        for _ in range(iters):
            y = self.solve(x)
            est = np.abs(y).sum()
            xi = np.where(y >= 0, 1.0, -1.0)
            z = self.solve(xi, trans=True)
            j = int(np.argmax(np.abs(z)))
            if np.abs(z[j]) <= z @ x:
                break
            x = np.zeros(n)
            x[j] = 1.0
        return float(anorm * est)


def solve_direct(band, n: int, k: int, b, trans: bool = False) -> np.ndarray:
    return DirectLU(band, n, k).solve(b, trans)


# ----------------------------------------------------------- partitioning

def partition(n: int, p: int):
    """Sec. 3.1: the first P_r = N - P*floor(N/P) blocks have floor(N/P)+1
    rows, the rest floor(N/P).  Returns (sizes, starts) as int64 arrays."""
    if p < 1 or p > n:
        raise ValueError("need 1 <= P <= N")
    q, pr = divmod(n, p)
    sizes = np.array([q + 1] * pr + [q] * (p - pr), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return sizes, starts


# ------------------------------------------------------- SaP preconditioner

FP64_EPS = 2.0 ** -52
FP32_EPS = 2.0 ** -23


@dataclass
class SapPrecond:
    """SaP-D / SaP-C preconditioner built from the paper's steps, float64.

    boost_eps: pivot-boost threshold factor; tau_i = boost_eps * max|A_i|
    (entrywise over the diagonal block).  boost_eps < 0 disables boosting.
    """

    band: np.ndarray
    n: int
    k: int
    p: int
    coupled: bool
    boost_eps: float = FP64_EPS
    sizes: np.ndarray = field(init=False)
    starts: np.ndarray = field(init=False)
    lu: list = field(init=False, default_factory=list)
    ul: list = field(init=False, default_factory=list)
    n_boosted: int = field(init=False, default=0)

    def __post_init__(self):
        self.band = _f64(self.band)
        n, k, p = self.n, self.k, self.p
        self.sizes, self.starts = partition(n, p)
        # with K = 0 there are no coupling blocks: SaP-C reduces to SaP-D
        self.cpl = self.coupled and p > 1 and k > 0
        if self.cpl and int(self.sizes.min()) < 2 * k:
            raise ValueError("coupled mode needs every block to have >= 2K rows")
        lib = _load()
        w = 2 * k + 1
        nb_tot = ctypes.c_int32(0)
        self.tau = []
        for i in range(p):
            nb, s0 = int(self.sizes[i]), int(self.starts[i])
            f = np.empty(nb * w, dtype=np.float64)
            lib.orc_block_load(n, k, _p(self.band), s0, nb, _p(f))
            tau = (self.boost_eps * lib.orc_block_maxabs(nb, k, _p(f))
                   if self.boost_eps >= 0 else -1.0)
            self.tau.append(tau)
            fu = f.copy() if self.cpl else None
            info = lib.orc_block_lu(nb, k, _p(f), tau, ctypes.byref(nb_tot))
            if info:
                raise np.linalg.LinAlgError("zero pivot %d in block %d" % (info - 1, i))
            self.n_boosted += nb_tot.value
            self.lu.append(f)
            if fu is not None:
                info = lib.orc_block_ul(nb, k, _p(fu), tau, ctypes.byref(nb_tot))
                if info:
                    raise np.linalg.LinAlgError("zero UL pivot %d in block %d" % (info - 1, i))
                self.n_boosted += nb_tot.value
                self.ul.append(fu)
        if self.cpl:
            self._tips()

    # -- factor-corner helpers (row window R(r,c) = f[r*w + c - r + k]) --
    def _rw(self, f, nb, r, c):
        return f[r * (2 * self.k + 1) + (c - r + self.k)]

    def _corner(self, f, nb, top: bool):
        """The K x K corner (top-left or bottom-right) of a block's row window."""
        k = self.k
        o = 0 if top else nb - k
        m = np.zeros((k, k))
        for a in range(k):
            for b in range(k):
                m[a, b] = self._rw(f, nb, o + a, o + b)
        return m

    def coupling_blocks(self, i: int):
        """B_i (super-diagonal, rows: last K of block i, cols: first K of
        block i+1) and C_{i+1} (sub-diagonal, rows: first K of block i+1,
        cols: last K of block i), Sec. 2.1 (0-based block index i)."""
        k, n, s = self.k, self.n, int(self.starts[i + 1])
        B = np.array([[band_get(self.band, n, k, s - k + a, s + b)
                       for b in range(k)] for a in range(k)])
        C = np.array([[band_get(self.band, n, k, s + a, s - k + b)
                       for b in range(k)] for a in range(k)])
        return B, C

    def _tips(self):
        """V_i^(b) = U_bb^{-1} L_bb^{-1} B_i from the bottom corners of LU(A_i);
        W_{i+1}^(t) = L'_tt^{-1} U'_tt^{-1} C_{i+1} from the top corners of
        UL(A_{i+1}); Rbar_i = I - W_{i+1}^(t) V_i^(b) and its LU with partial
        pivoting (eq:solveTopBottom)."""
        k = self.k
        self.B, self.C, self.V, self.W, self.Rbar, self.Rlu = [], [], [], [], [], []
        for i in range(self.p - 1):
            B, C = self.coupling_blocks(i)
            nb_i, nb_j = int(self.sizes[i]), int(self.sizes[i + 1])
            Mb = self._corner(self.lu[i], nb_i, top=False)
            L_bb = np.tril(Mb, -1) + np.eye(k)
            U_bb = np.triu(Mb)
            V = sla.solve_triangular(U_bb, sla.solve_triangular(
                L_bb, B, lower=True, unit_diagonal=True), lower=False)
            Mt = self._corner(self.ul[i + 1], nb_j, top=True)
            U_tt = np.triu(Mt, 1) + np.eye(k)
            L_tt = np.tril(Mt)
            W = sla.solve_triangular(L_tt, sla.solve_triangular(
                U_tt, C, lower=False, unit_diagonal=True), lower=True)
            Rbar = np.eye(k) - W @ V
            self.B.append(B); self.C.append(C); self.V.append(V); self.W.append(W)
            self.Rbar.append(Rbar)
            self.Rlu.append(sla.lu_factor(Rbar, check_finite=True))

    # -- block-diagonal solves, eq:diag-sys --
    def dinv(self, r, trans: bool = False) -> np.ndarray:
        g = np.array(r, dtype=np.float64, copy=True)
        lib = _load()
        for i in range(self.p):
            nb, s0 = int(self.sizes[i]), int(self.starts[i])
            seg = np.ascontiguousarray(g[s0:s0 + nb])
            lib.orc_block_solve(nb, self.k, _p(self.lu[i]), _p(seg), int(bool(trans)))
            g[s0:s0 + nb] = seg
        return g

    def reduced(self, g):
        """Truncated reduced solves (eq:solveTopBottom) for every interface:
        returns lists of x~^(t)_{i+1} and x~^(b)_i."""
        k = self.k
        xt_all, xb_all = [], []
        for i in range(self.p - 1):
            s = int(self.starts[i + 1])
            gb, gt = g[s - k:s], g[s:s + k]
            xt = sla.lu_solve(self.Rlu[i], gt - self.W[i] @ gb)
            xb = gb - self.V[i] @ xt
            xt_all.append(xt); xb_all.append(xb)
        return xt_all, xb_all

    def apply(self, r) -> np.ndarray:
        """z = M^{-1} r.  SaP-D: z = D^{-1} r (x ~ g, Sec. 2.1.1).  SaP-C:
        g = D^{-1} r, truncated reduced solves, then the purification solve
        A_i x_i = b_i - [C_i x~^(b)_{i-1}; 0; 0] - [0; 0; B_i x~^(t)_{i+1}]."""
        g = self.dinv(r)
        if not self.cpl:
            return g
        k = self.k
        xt_all, xb_all = self.reduced(g)
        rp = np.array(r, dtype=np.float64, copy=True)
        for i in range(self.p - 1):
            s = int(self.starts[i + 1])
            rp[s - k:s] -= self.B[i] @ xt_all[i]
            rp[s:s + k] -= self.C[i] @ xb_all[i]
        return self.dinv(rp)

    def apply_t(self, s) -> np.ndarray:
        """z = M^{-T} s, the exact transpose of ``apply``.  Writing
        M^{-1} = D^{-1}(I + Gamma Psi D^{-1}) with Psi the reduced solves and
        Gamma the coupling-block products, M^{-T} s = D^{-T}(s + Psi^T Gamma^T
        D^{-T} s)."""
        h = self.dinv(s, trans=True)
        if not self.cpl:
            return h
        k = self.k
        gbar = np.zeros(self.n)
        for i in range(self.p - 1):
            st = int(self.starts[i + 1])
            hb, ht = h[st - k:st], h[st:st + k]
            ybar = -(self.B[i].T @ hb)            # Gamma^T, bottom of block i
            zbar = -(self.C[i].T @ ht)            # Gamma^T, top of block i+1
            tbar = sla.lu_solve(self.Rlu[i], ybar - self.V[i].T @ zbar, trans=1)
            gbar[st:st + k] += tbar
            gbar[st - k:st] += zbar - self.W[i].T @ tbar
        return self.dinv(np.asarray(s, dtype=np.float64) + gbar, trans=True)


# ------------------------------------------------- rounding-error model (FP32)

def dinv_error_bound(M: "SapPrecond", r, u: float = 2.0 ** -24, blocks=None) -> np.ndarray:
    """First-order componentwise bound on |g_hat - g| for g = D^{-1} r when
    the block factorizations and the two triangular sweeps run in a format
    with unit roundoff u (FP32: 2^-24) and A and r are rounded to it.

    Standard backward-error results (Higham, Accuracy and Stability of
    Numerical Algorithms, 2nd ed., Thm 8.5 for triangular solves, Thm 9.3 and
    9.4 for LU without pivoting), with the inner-product length reduced to
    the K+1 terms a band row or column has: the computed g_hat solves
    (A_i + E_i) g_hat = r_i + dr_i with |dr_i| <= u|r_i| and
    |E_i| <= u|A_i| + gamma_m |L_i||U_i|, gamma_m = m u / (1 - m u),
    m = 3K + 8 (3(K+1) for the factorization and the two sweeps, plus the
    rounding of 1/u_jj and of the product by it, which the sweeps use).  To
    first order g_hat - g = A_i^{-1}(dr_i - E_i g), hence the bound
    |A_i^{-1}| (u|r_i| + (u|A_i| + gamma_m |L_i||U_i|) |g_i|), evaluated here
    with the FP64 factors and dense block inverses (small blocks only).  The
    order in which the sums are taken does not enter, so the bound covers
    any evaluation order of the same operations.  ``blocks`` limits the
    evaluation to those block indices (the other entries are NaN)."""
    k = M.k
    m = 3 * k + 8
    gam = m * u / (1.0 - m * u)
    r = np.asarray(r, dtype=np.float64)
    g = M.dinv(r)
    out = np.full(M.n, np.nan)
    w = 2 * k + 1
    for i in (range(M.p) if blocks is None else blocks):
        nb, s0 = int(M.sizes[i]), int(M.starts[i])
        f = M.lu[i].reshape(nb, w)
        L = np.eye(nb)
        U = np.zeros((nb, nb))
        A = np.zeros((nb, nb))
        b2 = M.band.reshape(2 * k + 1, M.n)
        for rr in range(nb):
            lo, hi = max(0, rr - k), min(nb, rr + k + 1)
            cs = np.arange(lo, hi)
            v = f[rr, cs - rr + k]
            L[rr, lo:rr] = v[:rr - lo]
            U[rr, rr:hi] = v[rr - lo:]
            A[rr, lo:hi] = b2[k + rr - cs, s0 + cs]
        gi = np.abs(g[s0:s0 + nb])
        v = u * np.abs(r[s0:s0 + nb]) + u * (np.abs(A) @ gi) + gam * (np.abs(L) @ (np.abs(U) @ gi))
        out[s0:s0 + nb] = np.abs(np.linalg.inv(A)) @ v
    return out


def dinv_error_sigma(M: "SapPrecond", r, u: float = 2.0 ** -24, blocks=None) -> np.ndarray:
    """Standard deviation of g_hat - g per component under the statistical
    rounding model (each rounding a relative error of variance u^2/3,
    independent of the others; Higham, op. cit., Sec. 2.8), applied to the
    same first-order expression as ``dinv_error_bound``:
    g_hat - g = A_i^{-1}(dr_i - E_i g) with E_i = dA_0 + dA_1 and the
    entry (j, c) of dA_1 a sum over t of l_jt u_tc times up to m = 3K + 8
    roundings.  Summing variances instead of magnitudes gives
      var = (u^2/3) (A_i^{-1})^2 [r^2 + (A_i)^2 g^2 + m (L_i)^2 (U_i)^2 g^2]
    with squares taken entrywise.  Worst-case signs (the bound above) grow
    with the factor growth of the block and become vacuous for weakly
    dominant blocks; this model stays within an order of magnitude of what
    an FP32 evaluation actually shows.  ``blocks`` as for
    ``dinv_error_bound``."""
    k = M.k
    m = 3 * k + 8
    r = np.asarray(r, dtype=np.float64)
    g = M.dinv(r)
    out = np.full(M.n, np.nan)
    w = 2 * k + 1
    for i in (range(M.p) if blocks is None else blocks):
        nb, s0 = int(M.sizes[i]), int(M.starts[i])
        f = M.lu[i].reshape(nb, w)
        L = np.eye(nb)
        U = np.zeros((nb, nb))
        A = np.zeros((nb, nb))
        b2 = M.band.reshape(2 * k + 1, M.n)
        for rr in range(nb):
            lo, hi = max(0, rr - k), min(nb, rr + k + 1)
            cs = np.arange(lo, hi)
            v = f[rr, cs - rr + k]
            L[rr, lo:rr] = v[:rr - lo]
            U[rr, rr:hi] = v[rr - lo:]
            A[rr, lo:hi] = b2[k + rr - cs, s0 + cs]
        g2 = g[s0:s0 + nb] ** 2
        v = r[s0:s0 + nb] ** 2 + (A ** 2) @ g2 + m * ((L ** 2) @ ((U ** 2) @ g2))
        out[s0:s0 + nb] = np.sqrt((u * u / 3.0) * ((np.linalg.inv(A) ** 2) @ v))
    return out


# --------------------------------------------------------------- BiCGStab(l)

@dataclass
class KrylovResult:
    x: np.ndarray
    iters: float               # Krylov-operator applications / (2l), in quarters for l=2
    converged: bool
    rel_resid_true: float
    rel_resid_precond: float
    restarts: int
    history: list              # (iters, preconditioned relative residual) at exit points


class Breakdown(RuntimeError):
    pass


def bicgstab_l(matvec, precond, b, tol: float = 1e-10, maxit: int = 500,
               ell: int = 2, reliable: float = 0.0, observe=None) -> KrylovResult:
    """Left-preconditioned BiCGStab(l) (Sleijpen & Fokkema 1993), x0 = 0.

    Solves M^{-1} A x = M^{-1} b.  Exit points follow every BiCG step j (after
    2j+1 of the 2l operator applications of one iteration) and the end of the
    minimal-residual part; for l = 2 they fall at quarters 1/4, 3/4 and 1.

    Stopping: when the recursive preconditioned residual drops below the
    current threshold, the true residual ||b - A x|| / ||b|| is computed; the
    solve stops if that is <= tol.  Otherwise the method restarts from the
    current x with the recomputed residual M^{-1}(b - A x) and rescales the
    threshold by ||M^{-1} t|| / ||t|| of that fresh residual t.

    reliable > 0 adds the reliable-update rule of Sleijpen and van der Vorst
    (1996): the same true-residual test and restart also happen once the
    recursive residual has dropped by the factor `reliable` since the last
    (re)start.  With a preconditioner applied in lower precision the recursive
    residual stops tracking the true one near that precision; restarting there
    lets the next steps reduce the true residual again.

    observe (test hook, read-only): called at every exit point, before its
    test, as observe(kind, napply, x, r, u) with kind "bicg" after a BiCG step
    and "mr" after the minimal-residual part; r and u are the current lists
    r_0..r_l and u_0..u_l (after the MR part, r_1..r_l are the vectors
    orthogonalized by modified Gram-Schmidt).  Copies are passed.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        return KrylovResult(x, 0.0, True, 0.0, 0.0, 0, [])

    def op(v):
        return precond(matvec(v))

    napply = 0
    restarts = 0
    history = []
    r0 = precond(b)
    pnorm0 = float(np.linalg.norm(r0))
    thr = tol * pnorm0

    def fresh_state(rvec):
        return dict(r=[rvec.copy()] + [None] * ell, u=[np.zeros(n)] + [None] * ell,
                    rt=rvec.copy(), rho0=1.0, alpha=0.0, omega=1.0)

    st = fresh_state(r0)
    rel_true = 1.0
    pnorm = pnorm0
    pstart = pnorm0

    def check():
        """Exit test at an exit point.  Returns True when converged."""
        nonlocal thr, st, napply, restarts, rel_true, x, pstart
        pn = float(np.linalg.norm(st["r"][0]))
        history.append((napply / (2 * ell), pn / pnorm0))
        if pn > thr and not (reliable > 0.0 and pn <= reliable * pstart):
            return False
        t = b - matvec(x)
        rel_true = float(np.linalg.norm(t)) / bnorm
        if rel_true <= tol:
            return True
        rfresh = precond(t)
        napply += 1
        restarts += 1
        tn = float(np.linalg.norm(t))
        pstart = float(np.linalg.norm(rfresh))
        thr = tol * bnorm * pstart / tn
        st = fresh_state(rfresh)
        return False

    for _it in range(maxit):
        r, u, rt = st["r"], st["u"], st["rt"]
        st["rho0"] = -st["omega"] * st["rho0"]
        restarted = False
        for j in range(ell):                                   # BiCG part
            rho1 = float(r[j] @ rt)
            if st["rho0"] == 0.0:
                raise Breakdown("rho0 = 0")
            beta = st["alpha"] * rho1 / st["rho0"]
            st["rho0"] = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = op(u[j]); napply += 1
            gamma = float(u[j + 1] @ rt)
            if gamma == 0.0:
                raise Breakdown("gamma = 0")
            st["alpha"] = st["rho0"] / gamma
            for i in range(j + 1):
                r[i] = r[i] - st["alpha"] * u[i + 1]
            x = x + st["alpha"] * u[0]
            if observe is not None:
                observe("bicg", napply, x.copy(), [None if v is None else v.copy() for v in r],
                        [None if v is None else v.copy() for v in u])
            if check():
                return KrylovResult(x, napply / (2 * ell), True, rel_true,
                                    float(np.linalg.norm(st["r"][0])) / pnorm0,
                                    restarts, history)
            if st["r"] is not r:          # restarted at this exit point
                restarted = True
                break
            r[j + 1] = op(r[j]); napply += 1
        if restarted:
            continue
        # minimal-residual part (modified Gram-Schmidt)
        tau = np.zeros((ell + 1, ell + 1))
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = float(r[j] @ r[i]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = float(r[j] @ r[j])
            if sigma[j] == 0.0:
                raise Breakdown("sigma = 0")
            gp[j] = float(r[0] @ r[j]) / sigma[j]
        g = np.zeros(ell + 1)
        g[ell] = gp[ell]
        st["omega"] = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1)
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            x = x + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        if observe is not None:
            observe("mr", napply, x.copy(), [v.copy() for v in r], [v.copy() for v in u])
        if check():
            return KrylovResult(x, napply / (2 * ell), True, rel_true,
                                float(np.linalg.norm(st["r"][0])) / pnorm0,
                                restarts, history)
    t = b - matvec(x)
    return KrylovResult(x, napply / (2 * ell), False,
                        float(np.linalg.norm(t)) / bnorm,
                        float(np.linalg.norm(st["r"][0])) / pnorm0, restarts, history)


# ------------------------------------------------------ conjugate gradient

def cg(matvec, precond, b, tol: float = 1e-10, maxit: int = 500,
       observe=None) -> KrylovResult:
    """Preconditioned conjugate gradient (Saad, Iterative Methods for Sparse
    Linear Systems, 2nd ed., Alg. 9.1), x0 = 0: the paper's outer loop when A
    is symmetric positive definite (Sec. 2.1.1).  r is the unpreconditioned
    residual b - A x, updated recursively; z = M^{-1} r.

    Stopping as in ``bicgstab_l``: when ||r|| <= tol ||b|| the true residual
    is computed; the solve stops if it meets the tolerance, otherwise CG
    restarts from the current x with r = b - A x (p = z = M^{-1} r).
    ``iters`` counts CG steps (products A p).  A step with p^T A p <= 0 (A
    or the preconditioned operator not positive definite) raises Breakdown.
    observe (test hook): called after every step as observe(it, x, r)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        return KrylovResult(x, 0.0, True, 0.0, 0.0, 0, [])
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rho = float(r @ z)
    restarts, history = 0, []
    rel_true = 1.0
    for it in range(1, maxit + 1):
        q = matvec(p)
        pq = float(p @ q)
        if not pq > 0.0:
            raise Breakdown("p^T A p <= 0")
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rn = float(np.linalg.norm(r))
        history.append((it, rn / bnorm))
        if observe is not None:
            observe(it, x.copy(), r.copy())
        if rn <= tol * bnorm:
            t = b - matvec(x)
            rel_true = float(np.linalg.norm(t)) / bnorm
            if rel_true <= tol:
                return KrylovResult(x, float(it), True, rel_true, rn / bnorm, restarts, history)
            r = t
            restarts += 1
            z = precond(r)
            p = z.copy()
            rho = float(r @ z)
            continue
        z = precond(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    t = b - matvec(x)
    return KrylovResult(x, float(maxit), False, float(np.linalg.norm(t)) / bnorm,
                        float(np.linalg.norm(r)) / bnorm, restarts, history)


def sap_solve_cg(band, n: int, k: int, b, p: int, coupled: bool, tol: float = 1e-10,
                 maxit: int = 500, boost_eps: float = FP64_EPS):
    """SaP preconditioner + CG on a symmetric positive definite A."""
    M = SapPrecond(band, n, k, p, coupled, boost_eps)
    res = cg(lambda v: bandmv(band, n, k, v), M.apply, b, tol, maxit)
    return res.x, res, M


# ------------------------------------------------------------ full solves

def sap_solve(band, n: int, k: int, b, p: int, coupled: bool, tol: float = 1e-10,
              maxit: int = 500, boost_eps: float = FP64_EPS,
              trans: bool = False):
    """SaP preconditioner + BiCGStab(2) on A x = b (trans: A^T x = b with
    M^{-T} as the preconditioner).  Returns (x, KrylovResult, SapPrecond)."""
    M = SapPrecond(band, n, k, p, coupled, boost_eps)
    if not trans:
        res = bicgstab_l(lambda v: bandmv(band, n, k, v), M.apply, b, tol, maxit)
    else:
        res = bicgstab_l(lambda v: bandmv(band, n, k, v, trans=True), M.apply_t,
                         b, tol, maxit)
    return res.x, res, M


# --------------------------------------------------------------- gradients

def band_grad(lam, x, n: int, k: int) -> np.ndarray:
    """dL/dA restricted to the band, in the band layout: entry (r, c) gets
    -lam_r * x_c for |r - c| <= K; padding slots are 0."""
    lam, x = np.asarray(lam), np.asarray(x)
    g = np.zeros((2 * k + 1, n))
    cols = np.arange(n)
    for q in range(2 * k + 1):
        d = q - k
        c = cols[max(0, -d):n - max(0, d)]
        g[q, c] = -lam[c + d] * x[c]
    return g.reshape(-1)


def gradients(band, n: int, k: int, b, x_target):
    """Loss L = 0.5 ||x - x_target||^2 with x = A^{-1} b.  Returns
    (x, dL/db = A^{-T}(x - x_target), dL/dA on the band)."""
    lu = DirectLU(band, n, k)
    x = lu.solve(b)
    lam = lu.solve(x - np.asarray(x_target), trans=True)
    return x, lam, band_grad(lam, x, n, k)
