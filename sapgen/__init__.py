"""Seeded synthetic workloads for the dense banded SaP solver.

This module is shared by the CPU oracle and by the GPU path's tests and
benchmark.  It only draws random numbers and lays them out; it performs none
of the solver's arithmetic.  The one product it forms, b = A x_true, is input
construction (the right-hand side of the test problem), done here with a
plain per-diagonal numpy expression.

Random numbers come from a counter-based generator: the SplitMix64 output
function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to an affine mix of (seed, stream, index).
Any single draw can therefore be regenerated without replaying a sequence.

Matrix recipe (the paper's dense experiments use random dense banded matrices
with a prescribed degree of diagonal dominance d, Sec. 2.1 eq:diagDominanceDef
and Sec. 4.1):

* off-diagonal a[r, c], 0 < |r - c| <= K, inside the matrix: U[-1, 1)
  from stream 0 at index r*(2K+1) + (c - r + K);
* a[r, r] = s_r * d * sum_{c != r} |a[r, c]|, with s_r = +1 or -1 from the
  sign of the stream-1 draw at index r (fair coin); for K = 0 (no
  off-diagonals) a[r, r] = s_r * d;
* optional row scaling: row r multiplied by 10**(2*u_r), u_r from stream 3,
  applied after the diagonal is set (so every row keeps its dominance d);
* symmetric variant (the SPD workload of the conjugate-gradient outer
  loop): a[r, c] = a[c, r] is the stream-0 draw of the lower entry,
  index max(r,c)*(2K+1) + (min(r,c) - max(r,c) + K), and the diagonal is
  +d * sum_{c != r} |a[r, c]| (no random sign): with d > 1 the matrix is
  symmetric and strictly diagonally dominant with a positive diagonal,
  hence positive definite;
* x_true ~ U[-1, 1) from stream 2; b = A x_true;
* x_target ~ N(0, 1) from stream 4 by the Box-Muller transform.

Band layout ("tall and thin" storage, Sec. 3.1 "Matrix storage"): an
N x (2K+1) array stored column-major, i.e. a flat array where storage column
q (0 <= q <= 2K) is contiguous and holds a[c + q - K, c] at position q*N + c.
The diagonal is storage column K.  Slots with c + q - K outside [0, N) are
padding; the generator fills them with ``pad`` (0 by default).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "STREAM_OFFDIAG", "STREAM_SIGN", "STREAM_XTRUE", "STREAM_ROWSCALE",
    "STREAM_XTARGET", "STREAM_PICK",
    "splitmix64_uniform", "band_index", "BandedProblem", "make_problem",
    "band_to_dense", "dense_to_band", "normal_draws", "WORKLOADS",
]

STREAM_OFFDIAG = 0
STREAM_SIGN = 1
STREAM_XTRUE = 2
STREAM_ROWSCALE = 3
STREAM_XTARGET = 4
STREAM_PICK = 5
STREAM_SPARSE = 6        # sparse workloads: pattern, values, permutations

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_SEED_MUL = np.uint64(0xD1B54A32D192ED03)
_STREAM_MUL = np.uint64(0x8CB92BA72F3D8DD7)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (variant 13 finalizer), elementwise on uint64."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def splitmix64_uniform(seed: int, stream: int, index) -> np.ndarray:
    """Uniform draws in [-1, 1) with 53 random bits, one per index.

    state = seed*C_seed + stream*C_stream + (index+1)*golden  (mod 2^64),
    value = mix64(state) >> 11, scaled to [0, 1) and mapped to [-1, 1).
    """
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = (np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * _SEED_MUL
                + np.uint64(stream) * _STREAM_MUL)
        state = base + (idx + np.uint64(1)) * _GOLDEN
    z = _mix64(state)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def normal_draws(seed: int, stream: int, n: int) -> np.ndarray:
    """N(0,1) draws by Box-Muller from pairs of uniforms (indices 2i, 2i+1)."""
    i = np.arange(n, dtype=np.uint64)
    u1 = 0.5 * (splitmix64_uniform(seed, stream, 2 * i) + 1.0)      # [0, 1)
    u2 = 0.5 * (splitmix64_uniform(seed, stream, 2 * i + 1) + 1.0)
    u1 = 1.0 - u1                                                     # (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def band_index(n: int, k: int, r, c):
    """Flat position of a[r, c] in the band layout (requires |r - c| <= k)."""
    return (k + np.asarray(r) - np.asarray(c)) * n + np.asarray(c)


@dataclass
class BandedProblem:
    n: int
    k: int
    d: float
    seed: int
    band: np.ndarray        # float64, (2k+1)*n, band layout
    x_true: np.ndarray      # float64, n
    b: np.ndarray           # float64, n
    row_scale: np.ndarray | None = None

    def band2d(self) -> np.ndarray:
        """View as (2k+1, n): row q is storage column q (a diagonal)."""
        return self.band.reshape(2 * self.k + 1, self.n)


def make_problem(n: int, k: int, d: float = 1.0, seed: int = 0,
                 row_scale_decades: float = 0.0, pad: float = 0.0,
                 with_rhs: bool = True, symmetric: bool = False) -> BandedProblem:
    """Build A (band layout), x_true and b = A x_true for one workload."""
    if symmetric and row_scale_decades > 0.0:
        raise ValueError("row scaling would break the symmetry")
    if n < 1 or k < 0 or k >= n:
        raise ValueError("need n >= 1 and 0 <= k < n")
    w = 2 * k + 1
    band = np.full((w, n), pad, dtype=np.float64)
    rowabs = np.zeros(n, dtype=np.float64)
    cols = np.arange(n, dtype=np.int64)
    for q in range(w):
        delta = q - k                     # row - col
        if delta == 0:
            continue
        c = cols[max(0, -delta):n - max(0, delta)]
        r = c + delta
        if symmetric:          # the draw of the lower entry (max(r,c), min(r,c))
            hi, lo = np.maximum(r, c), np.minimum(r, c)
            idx = hi * w + (lo - hi + k)
        else:
            idx = r * w + (c - r + k)
        vals = splitmix64_uniform(seed, STREAM_OFFDIAG, idx.astype(np.uint64))
        band[q, c] = vals
        rowabs[r] += np.abs(vals)
    sign = np.where(splitmix64_uniform(seed, STREAM_SIGN,
                                       np.arange(n, dtype=np.uint64)) < 0.0,
                    -1.0, 1.0)
    if symmetric:
        sign = np.ones(n)
    band[k, :] = sign * d * (rowabs if k > 0 else 1.0)
    scale = None
    if row_scale_decades > 0.0:
        u = splitmix64_uniform(seed, STREAM_ROWSCALE, np.arange(n, dtype=np.uint64))
        scale = 10.0 ** (row_scale_decades * u)
        for q in range(w):
            delta = q - k
            c = cols[max(0, -delta):n - max(0, delta)]
            band[q, c] *= scale[c + delta]
    x_true = splitmix64_uniform(seed, STREAM_XTRUE, np.arange(n, dtype=np.uint64))
    b = np.zeros(n, dtype=np.float64)
    if with_rhs:
        for q in range(w):
            delta = q - k
            c = cols[max(0, -delta):n - max(0, delta)]
            b[c + delta] += band[q, c] * x_true[c]
    return BandedProblem(n=n, k=k, d=d, seed=seed, band=band.reshape(-1),
                         x_true=x_true, b=b, row_scale=scale)


def band_to_dense(band: np.ndarray, n: int, k: int) -> np.ndarray:
    """Dense N x N copy of a band-layout matrix (padding slots ignored)."""
    b2 = np.asarray(band).reshape(2 * k + 1, n)
    a = np.zeros((n, n), dtype=b2.dtype)
    cols = np.arange(n)
    for q in range(2 * k + 1):
        delta = q - k
        c = cols[max(0, -delta):n - max(0, delta)]
        a[c + delta, c] = b2[q, c]
    return a


def dense_to_band(a: np.ndarray, k: int, pad: float = 0.0) -> np.ndarray:
    """Band layout of the entries |r - c| <= k of a dense matrix."""
    n = a.shape[0]
    b2 = np.full((2 * k + 1, n), pad, dtype=a.dtype)
    cols = np.arange(n)
    for q in range(2 * k + 1):
        delta = q - k
        c = cols[max(0, -delta):n - max(0, delta)]
        b2[q, c] = a[c + delta, c]
    return b2.reshape(-1)


@dataclass
class SparseProblem:
    n: int
    rowptr: np.ndarray      # int64, n+1
    colidx: np.ndarray      # int32, nnz (sorted within each row)
    vals: np.ndarray        # float64, nnz
    x_true: np.ndarray
    b: np.ndarray
    k0: int                 # half-bandwidth of the hidden banded matrix

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for r in range(self.n):
            lo, hi = self.rowptr[r], self.rowptr[r + 1]
            a[r, self.colidx[lo:hi]] = self.vals[lo:hi]
        return a


def _perm(seed: int, salt: int, n: int) -> np.ndarray:
    """A permutation of 0..n-1: the ranks of n uniform draws (index salt*n+i)."""
    u = splitmix64_uniform(seed, STREAM_SPARSE, salt * n + np.arange(n, dtype=np.uint64))
    return np.argsort(u, kind="stable").astype(np.int64)


def make_sparse_problem(n: int, k0: int, density: float = 0.3, d: float = 1.5,
                        seed: int = 0) -> SparseProblem:
    """A sparse system whose structure hides a banded, diagonally dominant
    matrix (the kind of input the reordering front end of Sec. 3.1 is for):

    * B: half-bandwidth k0; each off-diagonal slot (r, c), 0 < |r-c| <= k0,
      is a nonzero with probability `density` (stream 6, index
      r*(2 k0 + 1) + (c - r + k0), value mapped from [-1, 1)), its value the
      stream-0 draw of that slot; b_rr = s_r d sum|b_rc| as for the dense
      workloads (at least d if the row has no off-diagonal);
    * A = S R B S^T: R a random row permutation (moves the heavy diagonal off
      the diagonal), S a random symmetric permutation (scatters the band);
      both from stream 6 (salts 1 and 2);
    * x_true ~ U[-1, 1) (stream 2), b = A x_true."""
    w = 2 * k0 + 1
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for delta in range(-k0, k0 + 1):
        if delta == 0:
            continue
        c = np.arange(max(0, -delta), n - max(0, delta), dtype=np.int64)
        r = c + delta
        slot = r * w + (c - r + k0)
        keep = splitmix64_uniform(seed, STREAM_SPARSE, (slot + 3 * n).astype(np.uint64)) * 0.5 + 0.5 < density
        v = splitmix64_uniform(seed, STREAM_OFFDIAG, slot.astype(np.uint64))
        rows.append(r[keep]); cols.append(c[keep]); vals.append(v[keep])
        np.add.at(diag, r[keep], np.abs(v[keep]))
    sign = np.where(splitmix64_uniform(seed, STREAM_SIGN, np.arange(n, dtype=np.uint64)) < 0.0,
                    -1.0, 1.0)
    dval = sign * d * np.where(diag > 0, diag, 1.0)
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(dval)
    r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    R = _perm(seed, 1, n)          # row r of B becomes row R[r]
    S = _perm(seed, 2, n)          # index i becomes S[i] (rows and columns)
    r2 = S[R[r]]
    c2 = S[c]
    order = np.lexsort((c2, r2))
    r2, c2, v = r2[order], c2[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r2 + 1, 1)
    rowptr = np.cumsum(rowptr)
    x_true = splitmix64_uniform(seed, STREAM_XTRUE, np.arange(n, dtype=np.uint64))
    b = np.zeros(n)
    np.add.at(b, r2, v * x_true[c2])
    return SparseProblem(n=n, rowptr=rowptr, colidx=c2.astype(np.int32), vals=v,
                         x_true=x_true, b=b, k0=k0)


# The five workloads: sizes, dominance, partitions, mode and precisions.
WORKLOADS = {
    "sapd_n10k_k10": dict(n=10_000, k=10, d=1.0, p=16, mode="decoupled",
                          factor_prec="fp64", tol=1e-10, row_scale_decades=0.0),
    "sapc_n200k_k50": dict(n=200_000, k=50, d=1.0, p=64, mode="coupled",
                           factor_prec="fp64", tol=1e-10, row_scale_decades=0.0),
    "sapc_n500k_k200_mixed": dict(n=500_000, k=200, d=0.5, p=128, mode="coupled",
                                  factor_prec="fp32", tol=1e-10,
                                  row_scale_decades=0.0),
    "sapc_n100k_k32_adjoint": dict(n=100_000, k=32, d=1.0, p=32, mode="coupled",
                                   factor_prec="fp32", tol=1e-10,
                                   row_scale_decades=0.0),
    "sapc_n200k_k100_weak": dict(n=200_000, k=100, d=0.1, p=64, mode="coupled",
                                 factor_prec="fp32", tol=1e-8,
                                 row_scale_decades=2.0),
}

# Symmetric positive definite workloads for the conjugate-gradient outer loop
# (not among the five benchmark configurations): the benchmark's size and
# band with a symmetric, strictly dominant matrix.
SPD_WORKLOADS = {
    "spd_n200k_k50": dict(n=200_000, k=50, d=1.05, p=64, mode="decoupled",
                          factor_prec="fp64", tol=1e-10, row_scale_decades=0.0,
                          symmetric=True),
}
