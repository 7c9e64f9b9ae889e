/*
 * sap.h -- C ABI of the MI355X (gfx950) split-and-parallelize (SaP) solver
 * for dense banded linear systems A x = b.
 *
 * Method: Li, Serban and Negrut, "Analysis of a splitting approach for the
 * parallel solution of linear systems on GPU cards", arXiv:1509.07919.
 *   - Sec. 2.1 (eq:LeftRightSpikes, eq:diag-sys, eq:spike-sys,
 *     eq:SPIKE_reduced_system, eq:solveTopBottom and the purification
 *     equations): partition A into P diagonal blocks A_i, factor each, and
 *     couple neighbouring blocks through the truncated spike tips.
 *   - Sec. 2.1.1: decoupled (SaP-D, M = diag(A_i)) and coupled (SaP-C,
 *     truncated reduced system + purification) preconditioners inside an
 *     outer left-preconditioned BiCGStab(2).
 *   - Sec. 2.2, pivot-boosting paragraph: block LU/UL without pivoting; a
 *     pivot whose magnitude falls below a threshold is boosted.
 *   - Sec. 3.1: partition sizes, band storage, LU/UL factorizations and the
 *     mixed-precision strategy (single-precision preconditioner, double-
 *     precision Krylov loop).
 *
 * Conventions for every entry point
 *   - All vector and matrix pointers are DEVICE pointers (HIP device memory
 *     of the current device) unless marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it in order; entry points that must read a device
 *     scalar (sap_solve, sap_solve_adjoint, sap_handle_status) synchronise
 *     on that stream only.
 *   - Return value: SAP_OK (0), SAP_NOT_CONVERGED (1, a warning) or a
 *     negative error code.  On error, sap_last_error() gives a message for
 *     the calling thread.  No C++ exception ever crosses this boundary.
 *
 * Band layout of A (Sec. 3.1, "Matrix storage"): the N x (2K+1) "tall and
 * thin" array stored column-major.  As a flat array of (2K+1)*N doubles,
 * storage column q (0..2K) is contiguous and holds a[c+q-K][c] at index
 * q*N + c; the diagonal is storage column K.  Slots whose row c+q-K lies
 * outside [0, N) are padding: never read, may hold any value (even NaN).
 */
#ifndef SAP_H_
#define SAP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SAP_OK              0
#define SAP_NOT_CONVERGED   1   /* warning: x holds the last iterate      */
#define SAP_ERR_INVALID    -1   /* bad argument (see sap_last_error)       */
#define SAP_ERR_NOSPACE    -2   /* workspace smaller than required         */
#define SAP_ERR_HIP        -3   /* a HIP runtime call failed               */
#define SAP_ERR_BREAKDOWN  -4   /* BiCGStab(2): rho0, gamma or sigma = 0   */
#define SAP_ERR_SINGULAR   -5   /* zero pivot (boosting off) / singular    */
                                /* reduced matrix                          */
#define SAP_ERR_STATE      -6   /* call out of order (e.g. solve before    */
                                /* factor)                                 */

/* preconditioner mode, Sec. 2.1.1 */
#define SAP_DECOUPLED 0         /* SaP-D: M^{-1} = D^{-1}                    */
#define SAP_COUPLED   1         /* SaP-C: truncated spikes + purification    */

/* precision of factors, spike tips, reduced matrices and sweeps (Sec. 3.1,
 * "Mixed Precision Strategy").  The Krylov loop is always FP64. */
#define SAP_PREC_FP64 0
#define SAP_PREC_FP32 1

typedef struct sap_options {
    int64_t n;            /* matrix order N >= 1                            */
    int32_t k;            /* half-bandwidth K, 0 <= K < N, K <= 255         */
    int32_t p;            /* partitions P, 1 <= P <= N (SaP-C: N/P >= 2K)   */
    int32_t mode;         /* SAP_DECOUPLED or SAP_COUPLED                   */
    int32_t factor_prec;  /* SAP_PREC_FP64 or SAP_PREC_FP32                 */
    double  boost_eps;    /* pivot boost: tau_i = boost_eps * max|A_i|.      */
                          /*  0 -> unit roundoff of factor_prec (2^-52 or    */
                          /*  2^-23); < 0 disables boosting.                 */
    int32_t adjoint;      /* nonzero: also keep the transposed factor copies */
                          /*  needed by sap_solve_adjoint                    */
    int32_t sweep_chunks; /* chains per block in each triangular sweep:     */
                          /*  0 -> chosen by the library (chunked for       */
                          /*  K < 64 only), 1 -> one chain per block,       */
                          /*  >= 2 -> at most this many (each chunk then    */
                          /*  holds >= 64 rows) for K < 128, whose chunk    */
                          /*  transfer matrices sap_factor then forms       */
                          /*  (N K^2 FP64 FMA per factor array); one chain  */
                          /*  above; must be >= 0                           */
    int32_t nrhs;         /* right-hand sides sap_solve_batch may take at   */
                          /*  once, 0..64 (0 -> 1); the workspace grows     */
                          /*  with it                                       */
} sap_options;

typedef struct sap_stats {
    double  iters;             /* Krylov-operator applications / 4: BiCGStab(2)
                                  iterations in quarters (Sec. 4.1.1)          */
    double  rel_resid_true;    /* ||b - A x||_2 / ||b||_2 at exit             */
    double  rel_resid_precond; /* recursive ||M^{-1} r|| / ||M^{-1} b||        */
    int32_t converged;         /* 1 if rel_resid_true <= tol                  */
    int32_t n_boosted;         /* pivots boosted during sap_factor            */
    int32_t restarts;          /* restarts after a failed true-residual check */
    int32_t n_apply;           /* Krylov-operator applications                */
    float   t_factor_ms;       /* device time of the last sap_factor          */
    float   t_lu_ms;           /*   of which block LU/UL (T_LU)               */
    float   t_tips_ms;         /*   of which B/C, spike tips and reduced      */
                               /*   factorization (T_BC + T_SPK + T_LUrdcd)   */
    float   t_solve_ms;        /* device time of this solve (T_Kry)           */
} sap_stats;

typedef struct sap_handle_ *sap_handle;

/* Bytes of device workspace sap_create needs for these options.  Returns
 * SAP_ERR_INVALID for invalid options. */
int sap_workspace_bytes(const sap_options *opt, size_t *bytes /* host */);

/* Validate options, compute the partition (Sec. 3.1: the first
 * P_r = N - P*floor(N/P) blocks get floor(N/P)+1 rows, the rest floor(N/P))
 * and carve the caller's workspace.  `workspace` is device memory of at
 * least sap_workspace_bytes() bytes, 256-byte aligned, owned by the caller
 * and borrowed by the handle until sap_destroy.  The handle itself and a
 * small pinned host buffer are owned by the library.  No device work. */
int sap_create(const sap_options *opt, void *workspace, size_t ws_bytes,
               sap_handle *out /* host */);

/* Numeric factorization (Sec. 2.1 and 3.1): per-block max-norm, LU of every
 * A_i without pivoting but with pivot boosting, and for SaP-C the UL of
 * every A_i, the coupling blocks B_i, C_{i+1}, the spike tips
 *   V_i^(b)     = U_bb^{-1} L_bb^{-1} B_i        (bottom corners of LU(A_i))
 *   W_{i+1}^(t) = L'_tt^{-1} U'_tt^{-1} C_{i+1}  (top corners of UL(A_{i+1}))
 * and Rbar_i = I - W_{i+1}^(t) V_i^(b) with its inverse (LU with partial
 * pivoting).  `a_band` (N*(2K+1) doubles, band layout) is BORROWED: it is
 * read again by every solve and must stay unchanged until the next
 * sap_factor or sap_destroy.  May be called again with new values.
 * Enqueue-only: device-side failures (zero pivot with boosting off,
 * singular Rbar) are reported by the next solve or by sap_handle_status. */
int sap_factor(sap_handle h, const double *a_band, void *stream);

/* Solve A x = b with left-preconditioned BiCGStab(2) (Sleijpen-Fokkema),
 * x0 = 0, preconditioner from the last sap_factor.  Exit tests at the three
 * exit points per iteration; a candidate exit is accepted only when the true
 * relative residual ||b - A x||/||b|| <= tol, otherwise the iteration
 * restarts from the current x with the recomputed residual.  maxit bounds
 * the BiCGStab(2) iterations.  b and x: N doubles each, must not overlap.
 * b = 0 gives x = 0 with no iteration counted.  The factorization's status
 * and ||b|| are read at the first exit test (one host round trip fewer), so
 * b = 0 and SAP_ERR_SINGULAR come back after one quarter step of work.
 * Returns SAP_OK, SAP_NOT_CONVERGED (x = last iterate), SAP_ERR_BREAKDOWN,
 * SAP_ERR_SINGULAR or SAP_ERR_STATE.
 * `st` (host, nullable) receives the statistics. */
int sap_solve(sap_handle h, const double *b, double *x, double tol,
              int32_t maxit, void *stream, sap_stats *st);

/* ------------------------------------------------------------------------
 * Sparse front end (Sec. 3.1 "Diagonal Boosting" and "Bandwidth reduction",
 * Sec. 3.3, Sec. 3.4 T_DB, T_CM, T_Drop, T_Asmbl): reorder a sparse A so
 * that a dense band of half-bandwidth K carries it, build that band for the
 * SaP preconditioner, and solve with the full reordered matrix in the
 * Krylov products.  A_hat = P D_r Q A D_c P^T with Q the row permutation of
 * diagonal boosting (maximum prod |a_{i sigma_i}| as a minimum-cost perfect
 * bipartite matching with costs log a_i - log |a_ij|, eq:DBrelated; D_r, D_c
 * scale A_hat to an I-matrix: |diagonal| = 1, |off-diagonal| <= 1) and P
 * the Cuthill-McKee ordering of the structure of Q A + (Q A)^T.  Entries
 * farther than K from the diagonal are left out of the band (drop-off) but
 * stay in the Krylov product.  Not built: the third-stage reordering of the
 * diagonal blocks (it needs full spikes). */
typedef struct sap_sparse_ *sap_sparse;

/* Analyse A given as host CSR (rowptr: N+1 int64, rowptr[0] = 0,
 * non-decreasing; colidx: rowptr[N] int32 column indices in [0, N), each at
 * most once per row, any order; vals: finite doubles; explicit zeros are
 * not edges of the matching; 1 <= N < 2^31).  Violations return
 * SAP_ERR_INVALID.  db, cm: nonzero to apply diagonal boosting and
 * Cuthill-McKee.  drop_frac in [0, 1): K is the least half-bandwidth whose
 * outside entries carry at most drop_frac of sum |a_hat| (0: every entry in
 * the band).  The reorderings run on the host; the plan keeps the reordered
 * structure and work vectors in device memory it allocates.  Returns
 * SAP_ERR_SINGULAR if A has no perfect matching (structurally singular). */
int sap_sparse_create(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                      const double *vals, int32_t db, int32_t cm, double drop_frac,
                      sap_sparse *out);

/* The plan's K (after drop-off) and the half-bandwidth without drop-off;
 * the maps (row r of A is row new_row[r] of A_hat; column c is column
 * new_col[c]) and the scales D_r, D_c (host arrays of N; any pointer may be
 * NULL). */
int sap_sparse_info(sap_sparse sp, int32_t *k, int32_t *k_full, int32_t *new_row,
                    int32_t *new_col, double *row_scale, double *col_scale);

/* Host time of the three analysis stages of sap_sparse_create, the sparse
 * front end's share of the time buckets of Sec. 3.4: the matching with its
 * scaling (T_DB), Cuthill-McKee (T_CM), and forming the reordered structure
 * with the drop-off K (T_Drop), in ms.  Any pointer may be NULL. */
int sap_sparse_times(sap_sparse sp, double *t_db_ms, double *t_cm_ms, double *t_drop_ms);

/* On the GPU: the values of A_hat from A's values (device array in the
 * original CSR order, same structure as at sap_sparse_create) and the band
 * of A_hat (device, (2K+1)*N doubles, band layout, padding zero) to hand to
 * sap_factor of a handle with this N and K.  Enqueue-only. */
int sap_sparse_assemble(sap_sparse sp, const double *vals, double *band, void *stream);

/* Solve A x = b (b, x device N-vectors in A's original order) with
 * BiCGStab(2) on A_hat y = b_hat, the preconditioner of h (factored on the
 * band from sap_sparse_assemble) and the sparse product of A_hat; then
 * x = D_c P^T y.  h must have the plan's N and K.  As sap_solve otherwise
 * (st->rel_resid_true refers to A_hat y = b_hat). */
int sap_solve_sparse(sap_handle h, sap_sparse sp, const double *b, double *x, double tol,
                     int32_t maxit, void *stream, sap_stats *st);

int sap_sparse_destroy(sap_sparse sp);

/* Solve A X = B for m right-hand sides at once (Sec. 4.1.1 discusses the
 * factorization cost that several right-hand sides share), 1 <= m <= nrhs
 * of the handle.  B and X are N x m, column-major (column c at + c*N), and
 * must not overlap.  One factorization serves all columns: the banded SpMV
 * reads A once per 4 columns, and for K <= 56 the triangular sweeps read
 * each factor row once per 4 columns; wider bands sweep the columns one
 * after another.  Every column runs BiCGStab(2) as sap_solve does, with its
 * own scalars, in lockstep with the others: a converged column is frozen,
 * and when a candidate exit of some column fails its true-residual test,
 * all active columns restart from their true residuals (so iteration counts
 * can differ from single solves; each converged column meets tol).  st
 * (host, nullable) receives m statistics records.  Returns SAP_OK when
 * every column converged, else as sap_solve. */
int sap_solve_batch(sap_handle h, const double *B, double *X, int32_t m,
                    double tol, int32_t maxit, void *stream, sap_stats *st);

/* Solve A x = b for symmetric positive definite A with the preconditioned
 * conjugate gradient method (the paper's outer loop when A is SPD,
 * Sec. 2.1.1; Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.1),
 * x0 = 0, preconditioner from the last sap_factor (SaP-D keeps M symmetric
 * up to rounding; SaP-C's truncated M is not symmetric, and CG then has no
 * convergence guarantee).  The residual b - A x is updated in FP64; when its
 * norm reaches tol ||b|| the true residual is tested, and CG restarts from
 * it if the test fails.  st->iters counts CG steps (products A p), n_apply
 * preconditioner applications.  p^T A p <= 0 returns SAP_ERR_BREAKDOWN (A
 * not positive definite).  Otherwise as sap_solve. */
int sap_solve_cg(sap_handle h, const double *b, double *x, double tol,
                 int32_t maxit, void *stream, sap_stats *st);

/* Adjoint solve A^T lambda = g with the same Krylov method, the transposed
 * banded SpMV and the exact transpose M^{-T} of the preconditioner built by
 * sap_factor (its factors and tips, no refactorization).  Needs
 * opt.adjoint != 0 at sap_create.  Same conventions as sap_solve. */
int sap_solve_adjoint(sap_handle h, const double *g, double *lambda,
                      double tol, int32_t maxit, void *stream, sap_stats *st);

/* Band of dL/dA = -lambda x^T: writes g_band[(K+r-c)*N + c] = -lambda_r x_c
 * for every band slot inside the matrix and 0 into padding slots.  With
 * lambda = A^{-T} dL/dx this is the gradient of L(x(A)) restricted to the
 * band; dL/db is lambda itself.  g_band: (2K+1)*N doubles. */
int sap_band_grad(sap_handle h, const double *lambda, const double *x,
                  double *g_band, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): sap_factor and
 * sap_solve of A x = b in one call, with the factors, tips, Krylov vectors
 * and every other intermediate in a static device array of
 * SAP_NOALLOC_SCRATCH_BYTES bytes inside the library instead of a caller
 * workspace.  Each GPU the library runs on holds one such array from the
 * first call on it until the process ends.  The call creates no handle,
 * event or stream and calls no allocation routine; it returns once x is
 * written (it synchronises `stream`).  opt as for sap_create, with
 * opt->adjoint = 0; a_band (borrowed only during the call), b and x as for
 * sap_factor and sap_solve.  Options whose workspace does not fit the array
 * (sap_workspace_bytes + 256 > SAP_NOALLOC_SCRATCH_BYTES) return
 * SAP_ERR_NOSPACE before any device work.  The statistics carry no device
 * times (t_*_ms = 0).  All calls on one GPU share its array and it keeps the
 * last call's contents: calls that overlap on one GPU (other host threads,
 * other streams) race and must be serialised by the caller. */
#define SAP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sap_solve_noalloc(const sap_options *opt, const double *a_band,
                      const double *b, double *x, double tol, int32_t maxit,
                      void *stream, sap_stats *st);

/* Device-side status of the last factorization, synchronising `stream`:
 * SAP_OK or SAP_ERR_SINGULAR; n_boosted (host, nullable) gets the number of
 * boosted pivots. */
int sap_handle_status(sap_handle h, void *stream, int32_t *n_boosted);

/* Single steps of the hot path, for parity testing and benchmarking.
 *   sap_spmv:          y = A v (trans = 0) or A^T v (trans = 1), FP64.
 *   sap_precond_apply: z = M^{-1} r (trans = 0) or M^{-T} r (trans = 1),
 *                      r and z FP64, arithmetic in the factor precision.
 * Both need a completed sap_factor; v/y and r/z must not overlap. */
int sap_spmv(sap_handle h, const double *v, double *y, int32_t trans,
             void *stream);
int sap_precond_apply(sap_handle h, const double *r, double *z,
                      int32_t trans, void *stream);

/* Copy the SaP-C interface matrices of interface i (0 <= i < P-1, between
 * blocks i and i+1) into host arrays of K*K doubles, row-major: V_i^(b),
 * W_{i+1}^(t) and Rbar_i.  Any pointer may be NULL.  Synchronises. */
int sap_get_tips(sap_handle h, int32_t i, double *v, double *w, double *rbar,
                 void *stream);

/* Copy rows j0 .. j0+count-1 of one factor coefficient array to the host,
 * widened to double, K+1 entries per row (row-major), for checking the
 * block LU of Sec. 3.1 directly.  which = 0: Lc, row j = [1, l(j+1,j) ..
 * l(j+K,j)] (column j of L); 1: Uc, row j = [1/u(j,j), u(j-1,j) ..
 * u(j-K,j)] (column j of U); 2: Lr, row j = [1, l(j,j-1) .. l(j,j-K)];
 * 3: Ur, row j = [1/u(j,j), u(j,j+1) .. u(j,j+K)] (2 and 3 need
 * adjoint = 1).  Entries that would leave the diagonal block are 0.  Needs
 * a completed sap_factor; synchronises. */
int sap_get_factor_rows(sap_handle h, int32_t which, int64_t j0, int64_t count,
                        double *out /* host */, void *stream);

/* The paper's split of the SaP-C preprocessing after the block LU (Sec.
 * 3.4): T_BC (gathering B_i and C_i), T_SPK (the spike tips V_i, W_i) and
 * T_LUrdcd (Rbar_i and its factorization), in milliseconds, of the last
 * sap_factor, into ms[0..2] (host).  Where the three run as separate
 * launches (large K) they are timed with events between them; where one
 * kernel does all three, its event time is split in proportion to the time
 * its workgroups spend in each phase (constant-rate device clock).  They are
 * recorded only while sap_profile is on (SAP_ERR_STATE otherwise).  Zero for
 * SaP-D.  Synchronises. */
int sap_tips_phase_times(sap_handle h, double *ms /* host[3] */, void *stream);

/* Per-kernel device timing, for benchmarking.  sap_profile(h, 1) resets the
 * counters and starts bracketing every kernel launch of the handle with a
 * pair of HIP events on the launch stream; sap_profile(h, 0) stops.
 * sap_kernel_time synchronises on the recorded events and returns the
 * summed device milliseconds and the number of launches of one kernel class
 * since the reset.  Recording adds event records between launches but does
 * not change the kernels. */
#define SAP_KERNEL_NORM    0   /* per-block max-norm                         */
#define SAP_KERNEL_LU      1   /* banded LU (and UL) of the diagonal blocks  */
#define SAP_KERNEL_TIPS    2   /* coupling blocks, spike tips, Rbar inverse  */
#define SAP_KERNEL_SWEEP   3   /* one triangular sweep over all blocks       */
#define SAP_KERNEL_CORR    4   /* SaP-C interface correction                 */
#define SAP_KERNEL_SPMV    5   /* banded SpMV (A or A^T, plain or residual)  */
#define SAP_KERNEL_KRYLOV  6   /* BiCGStab(2) dots and fused vector updates  */
#define SAP_KERNEL_XFER    7   /* chunk transfer matrices of the sweeps      */
#define SAP_KERNEL_COUNT   8
int sap_profile(sap_handle h, int32_t enable);
int sap_kernel_time(sap_handle h, int32_t kernel, double *ms /* host */,
                    int64_t *launches /* host */);

/* Release the handle (not the caller's workspace or matrix). */
int sap_destroy(sap_handle h);

/* Message for the last error status returned on this thread. */
const char *sap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SAP_H_ */
