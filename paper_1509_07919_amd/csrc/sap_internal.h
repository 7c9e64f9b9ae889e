// Internal declarations shared by the HIP translation units of libsap.
//
// Device data layout (all arrays live in the caller's workspace):
//
//   factor coefficient arrays, one row of CP entries per matrix column/row
//   j (global index), type T = float or double, CP = coef_pitch(K, sizeof T):
//     Lc[j*CP + 0] = 1,        Lc[j*CP + m] = l(j+m, j)   (column j of L)
//     Uc[j*CP + 0] = 1/u(j,j), Uc[j*CP + m] = u(j-m, j)   (column j of U)
//     Ur[j*CP + 0] = 1/u(j,j), Ur[j*CP + m] = u(j, j+m)   (row j of U)
//     Lr[j*CP + 0] = 1,        Lr[j*CP + m] = l(j, j-m)   (row j of L)
//   for m = 1..K, with 0 wherever j+m or j-m leaves the diagonal block, and
//   slots K+1..CP-1 zero (cleared when the handle first factors, never
//   written again).  Each row holds exactly the coefficients one step of a
//   forward or backward sweep pushes to its K successors, so every sweep
//   streams one contiguous run of rows; CP makes every row start on a
//   16-byte boundary and leaves at least one zero slot after the K
//   coefficients.  Ur/Lr exist only when the handle keeps the transposed
//   factors for the adjoint solve.
//
//   ULcorner[i*K*K + a*K + b]: bottom-right K x K corner of LU(J A_i J)
//   (unit-lower part below the diagonal, upper part with the pivots on and
//   above it); J reverses the order of the block's rows and columns, so this
//   is the top-left corner of the UL factorization of A_i read backwards.
//
//   interface arrays for SaP-C, i = 0..P-2, each K x K row-major, type T:
//   B, C (coupling blocks), V (= V_i^(b)), W (= W_{i+1}^(t)), Rbar, Rinv.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sap.h"

#include <string>

namespace sap {

constexpr int kMaxK = 255;
constexpr size_t kMaxLds = 160 * 1024;    // LDS bytes per workgroup on gfx950
constexpr int kDotBlocks = 512;   // fixed grid of the reduction kernels
constexpr int kMultiRhs = 4;      // right-hand sides per workgroup in multi-RHS kernels
constexpr int kMaxRhs = 64;       // right-hand sides per batched solve

// row pitch (entries) of the factor coefficient arrays: K + 1 coefficients,
// at least one zero, rounded up to a multiple of 16 bytes
__host__ __device__ inline int coef_pitch(int k, int tsize)
{
    const int per16 = 16 / tsize;
    return (k + 2 + per16 - 1) / per16 * per16;
}

enum KrylovOp : int {
    OP_INIT = 0,   // d0=(r0,rt) d1=(r0,r0): rho=1,alpha=0,omega=1 then j=0 prep
    OP_GAMMA,      // d0=(u_{j+1},rt): alpha = rho0/gamma
    OP_EXIT,       // d0=(r0,r0): publish ||r0||^2
    OP_RHO,        // d0=(r_j,rt): beta = alpha*rho1/rho0, rho0 = rho1
    OP_MR1,        // d0=(r1,r1) d1=(r0,r1) d2=(r2,r1)
    OP_MR2,        // d0=(r2,r2) d1=(r0,r2)
    OP_FINAL,      // d0=(r0,r0) d1=(r0,rt): publish, then next j=0 prep
    OP_NORM,       // d0=(v,v): publish only
    OP_TRUE,       // d0=(t,t): the true residual at a restart, to host slot H_TRUE
    OP_SPEC,       // d0=(t,t): the true residual ahead of an exit test, to H_SPEC
    OP_BNORM,      // d0=(b,b): the right-hand side's squared norm, to H_BNORM
    // preconditioned conjugate gradient (SPD A)
    OP_CG_INIT,    // d0=(r,z) d1=(r,r): rho = (r,z), publish ||r||^2
    OP_CG_ALPHA,   // d0=(p,Ap): alpha = rho / (p,Ap), breakdown unless > 0
    OP_CG_BETA,    // d0=(r,z): beta = (r,z) / rho, rho = (r,z)
};

// device scalar slots of the BiCGStab(2) recurrences (double sc[kScalars])
enum ScalarSlot : int {
    S_RHO0 = 0, S_ALPHA, S_OMEGA, S_BETA, S_GAMMA, S_SIGMA1, S_SIGMA2,
    S_GP1, S_GP2, S_TAU12, S_G1, S_G2, S_GPP1, S_NRM2, S_BREAK, kScalars = 32
};

// host-visible (pinned, mapped) result slots written by reduction kernels
// H_NRM0: squared norm of the (re)started preconditioned residual (OP_INIT);
// H_TRUE: squared norm of the true residual a restart started from (OP_TRUE);
// H_NBOOST, H_SING: the factorization's status words (DotArgs::status);
// H_SPEC: squared norm of the true residual enqueued ahead of an exit test;
// H_BNORM: squared norm of the right-hand side (OP_BNORM)
enum HostSlot : int { H_NRM2 = 0, H_BREAK = 1, H_NRM0 = 2, H_TRUE = 3, H_NBOOST = 4, H_SING = 5,
                      H_SPEC = 6, H_BNORM = 7, kHostSlots = 8 };

struct Partition {
    const int64_t *starts;   // P+1 block boundaries (device)
    int64_t n;
    int k;
    int p;
    int64_t maxnb;
};

// ------------------------------------------------------------- factorization
constexpr int kStatusWords = 16;   // int status[16]: [0] boosted pivots, [1] singular flag
hipError_t launch_block_norm(const double *band, const Partition &pt,
                             double *partial, int nchunk, int *status, hipStream_t s);

template <typename T>
struct LuArgs {
    const double *band;
    Partition pt;
    const double *partial;   // per-block norm partials [p][nchunk]
    int nchunk;
    double boost_eps;        // < 0: no boosting
    T *Lc, *Uc, *Lr, *Ur;    // Lr/Ur may be null
    T *corner;               // [p][K*K], UL direction only (may be null)
    int *status;             // [0] boosted pivots, [1] singular flag
    int with_ul;             // grid = 2P: blocks >= P run the UL direction
    double *wide;            // FP64 K > 160: one window slab per workgroup
};
template <typename T>
hipError_t launch_banded_lu(const LuArgs<T> &a, hipStream_t s);
// blocked LU with matrix-core trailing updates (used for K >= 64)
template <typename T>
hipError_t launch_lu_mfma(const LuArgs<T> &a, hipStream_t s);
bool lu_mfma_supported(int k, bool fp32);
// FP64 factors of bands wider than the register windows (K > 160): the
// window in a workspace slab of lu_wide_window_bytes(K) per workgroup
constexpr int kLuWideMinK = 161;
size_t lu_wide_window_bytes(int k);
hipError_t launch_lu_wide(const LuArgs<double> &a, double *slabs, hipStream_t s);

template <typename T>
struct TipsArgs {
    const double *band;
    Partition pt;
    const T *Lc, *Uc, *corner;
    T *B, *C, *V, *W, *Rbar, *Rlu, *Rinv;
    int *piv;
    int *status;
    unsigned long long *ticks;   // [3] per-phase workgroup time (LDS form), or null
};
// ev: 4 events (nullable) around the phases, see k_tips.hip
template <typename T>
hipError_t launch_tips(const TipsArgs<T> &a, hipStream_t s, hipEvent_t *ev = nullptr);
// whether the tips of this K and precision run as the single LDS kernel
bool tips_in_lds(int k, bool fp32);

// ------------------------------------------------------------------ sweeps
// One triangular sweep per diagonal block.  fwd: steps j = 0..nb-1 pushing
// to j+m; otherwise j = nb-1..0 pushing to j-m.  diag: multiply by F[j][0].
// Input: xin (double) or tin (T), plus optional boundary deltas (T) added to
// the top/bottom K rows of each block.  Output: dout (double) or tout (T).
//
// Chunked sweeps.  With nch >= 2 each block is cut into row chunks
// [c*clen, min((c+1)*clen, nb)) and one dependent chain runs per chunk.
// The state a chain hands to the next chunk (in its direction) is the
// vector of K pending sums p for the K rows that follow the chunk; it is
// linear in the chunk's inputs and in the state it received, so
//     p_out(c) = q(c) + X(c) p_in(c),
// where q(c) is the output state for a zero incoming state and X(c) is the
// K x K transfer matrix of the chunk (inputs zero), computed once per
// factorization.  A sweep then runs in two launches: phase 1 runs every
// chunk with a zero incoming state and writes q; phase 2 obtains each
// chunk's true incoming state by chaining the recurrence from the block's
// first chunk (K <= 56: every workgroup for its own chunk, at its start;
// larger K: the last phase-1 workgroup of each block, through st) and
// reruns the chunk from it, writing the outputs.
// Storage: q (type T), st (FP64) [p][nch][K]; X (FP64) [p][nch][K][K] with
// X[c][i][m] = d p_out[m] / d p_in[i] (row i contiguous in m); ticket [p]
// (zero between launches).  The states are chained in FP64 for either factor
// precision: with weak diagonal dominance the transfer matrices and the two
// terms of a link can exceed the state they form by orders of magnitude.
enum SweepPhase : int { SWEEP_WHOLE = 0, SWEEP_ZERO_STATE = 1, SWEEP_FROM_STATE = 2 };

template <typename T>
struct SweepArgs {
    const T *F;
    Partition pt;
    int fwd, diag;
    const double *xin;
    const T *tin;
    const T *dtop, *dbot;    // [p][K] or null
    double *dout;
    T *tout;
    int phase;               // SweepPhase
    int nch, clen;           // chunks per block (grid p*nch), rows per chunk
    T *q;                    // zero-state outgoing states [p][nch][K]
    double *st;              // chained entering states [p][nch][K] (FP64)
    const double *xf;        // transfer matrices (FP64 for either precision)
    unsigned *ticket;
    // From-state pass of a forward sweep (K <= 56): dtop enters as the
    // incoming state -dtop of each block's first chunk instead of being added
    // to its first K inputs (the same sums), so the zero-state pass of an
    // earlier sweep of the same input without dtop supplies q.
    int top_as_state;
    // right-hand sides (columns of xin/tin/dout/tout with leading dimension
    // ldv; dtop/dbot, q and st hold one slab per column).  m > 1 needs
    // K <= 56 (the circular kernels).
    int m;
    int64_t ldv;
};
template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &a, hipStream_t s);
// whether the chunked sweeps take dtop as an incoming state (top_as_state)
bool sweep_top_state_supported(int k);

// Transfer matrices X(c) of every chunk that hands a state on (see above),
// for up to four coefficient arrays in one launch.
template <typename T>
struct XferArgs {
    Partition pt;
    int nch, clen;
    int narr;
    const T *F[4];
    double *xf[4];           // FP64 whatever T is
    int fwd[4], diag[4];
    double *scratch;         // [narr][p][nch][2][K][K]: partial transfers X_2, X_3
};
template <typename T>
hipError_t launch_sweep_xfer(const XferArgs<T> &a, hipStream_t s);
// true when chunked sweeps are implemented for this K and precision
bool sweep_chunking_supported(int k, bool fp32);

// SaP-C interface correction: from g (T, full vector) compute the deltas
// added to the top (dtop) and bottom (dbot) K rows of each block before the
// purification sweep.  trans selects the exact transpose.
template <typename T>
struct CorrArgs {
    Partition pt;
    const T *g;
    const T *B, *C, *V, *W, *Rinv;
    T *dtop, *dbot;
    int trans;
    int m;                   // right-hand sides: g columns ld ldg apart,
    int64_t ldg;             // dtop/dbot one [p][K] slab per column
};
template <typename T>
hipError_t launch_correction(const CorrArgs<T> &a, hipStream_t s);

// ------------------------------------------------------------- SpMV / misc
// y = A v (trans 0) or A^T v; if b != null: y = b - A v (residual form).
hipError_t launch_spmv(const double *band, int64_t n, int k, const double *v,
                       const double *b, double *y, int trans, hipStream_t s);
// the same for m column-major right-hand sides (leading dimension n), read
// band entries serving kMultiRhs columns at once
hipError_t launch_spmv_multi(const double *band, int64_t n, int k, const double *v,
                             const double *b, double *y, int trans, int m, hipStream_t s);
hipError_t launch_band_grad(int64_t n, int k, const double *lam,
                            const double *x, double *g, hipStream_t s);

// ---------------------------------------------------------------- Krylov
struct DotArgs {
    const double *x[3];
    const double *y[3];
    int nd;
    int64_t n;
    double *partial;         // [kDotBlocks][3]
    double *sc;              // device scalars
    double *host;            // mapped pinned host slots (may be null)
    const int *status;       // if set, copied to host slots H_NBOOST, H_SING
    int op;
    // several right-hand sides: column c of every vector at c * ld; its
    // partials at partial + c*kDotBlocks*3, scalars at sc + c*kScalars, host
    // slots at host + c*kHostSlots; frozen columns (bit c, c < 64) are left
    // alone.  m = 0 means 1.
    int m;
    int64_t ld;
    uint64_t frozen;
};
hipError_t launch_dots(const DotArgs &a, hipStream_t s);

// Fused vector updates of BiCGStab(2) (l = 2), each optionally followed by
// dots handled as in launch_dots.
enum UpdKind : int {
    UPD_U0 = 0,      // u0 = r0 - beta u0
    UPD_J0,          // r0 -= alpha u1; x += alpha u0
    UPD_U01,         // u0 = r0 - beta u0; u1 = r1 - beta u1
    UPD_J1,          // r0 -= alpha u1; r1 -= alpha u2; x += alpha u0
    UPD_MR2,         // r2 -= tau12 r1
    UPD_FINAL,       // x += g1 r0 + gpp1 r1; r0 -= gp2 r2 + gp1 r1;
                     // u0 -= g2 u2 + g1 u1
    UPD_RESTART,     // rt = r0; u0 = 0
    // conjugate gradient: r = r0, z = r1, p = u0, q = A p = u1
    UPD_CG_INIT,     // p = z; dots (r,z), (r,r)
    UPD_CG_XR,       // x += alpha p; r -= alpha q; dot (r,r)
    UPD_CG_P,        // p = z + beta p
};
struct UpdArgs {
    int kind;
    int64_t n;
    double *x, *r0, *r1, *r2, *u0, *u1, *u2, *rt;
    DotArgs dots;            // dots.nd == 0: none
};
hipError_t launch_update(const UpdArgs &a, hipStream_t s);

hipError_t launch_fill(double *v, double val, int64_t n, hipStream_t s);

// ------------------------------------------------------------- sparse A
// A reordered sparse matrix on the device (CSR), for the Krylov product
struct CsrDev {
    int64_t n, nnz;
    const int64_t *rowptr;
    const int32_t *colidx;
    const double *vals;
};
hipError_t launch_csr_spmv(const CsrDev &m, const double *v, const double *b, double *y,
                           hipStream_t s);
hipError_t launch_map_vec(const double *in, const int32_t *map, const double *scale, double *out,
                          int64_t n, int gather, hipStream_t s);
// records an error for sap_last_error and returns code (sap_api.hip)
int api_fail(int code, const std::string &msg);
// the plan's device pieces (sparse_front.hip); false before sap_sparse_assemble
bool sparse_plan_parts(sap_sparse p, CsrDev *m, double **bhat, double **yhat,
                       const int32_t **new_row, const int32_t **new_col, const double **rs,
                       const double **cs);
int sparse_plan_k(sap_sparse p);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);   // bytes % 4 == 0
hipError_t launch_partition_starts(int64_t *starts, int64_t n, int p, hipStream_t s);

}  // namespace sap
