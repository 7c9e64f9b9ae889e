/*
 * CPU oracle for the dense banded SaP solver -- test infrastructure only.
 *
 * Plain, sequential, double-precision C.  Only the test suite, the package's
 * smoke check and the benchmark's CPU-baseline leg load this file's shared
 * library; the GPU library never does, and shares no code with it.
 *
 * Contents
 *   orc_bandmv          y = A v or A^T v straight from the band layout.
 *   orc_gb_factor/solve banded LU WITH partial pivoting (the plain definition
 *                       of solving A x = b; U grows to bandwidth 2K) and the
 *                       solves with A and A^T.
 *   orc_block_lu        LU of one diagonal block WITHOUT pivoting, with pivot
 *                       boosting (Sec. 2.2, pivot-boosting paragraph; Sec. 3.1
 *                       "LU/UL factorizations").
 *   orc_block_ul        the UL factorization of a block, eliminating from the
 *                       bottom row upward (Sec. 2.1, the paragraph after the
 *                       purification equations).
 *   orc_block_solve     D_i^{-1} and D_i^{-T} with the block's LU factors
 *                       (forward elimination / back substitution, Sec. 3.1).
 *
 * Band layout of A (Sec. 3.1 "Matrix storage"): a[r][c] with |r-c| <= K sits
 * at band[(K + r - c) * N + c]; other slots are padding and are never read.
 *
 * Block factor storage used here: a row-major "row window" R with
 * R(r, c) = f[r * (2K+1) + (c - r + K)] for |r - c| <= K, local indices.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ SpMV */

/* y = A v (trans = 0) or y = A^T v (trans = 1), from the definition
 * y_r = sum_c a[r][c] v_c over the band. */
void orc_bandmv(int64_t n, int32_t k, const double *band, const double *v,
                double *y, int32_t trans)
{
    for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        int64_t c0 = r - k < 0 ? 0 : r - k;
        int64_t c1 = r + k > n - 1 ? n - 1 : r + k;
        for (int64_t c = c0; c <= c1; ++c) {
            double a = band[(int64_t)(k + r - c) * n + c];
            if (!trans) y[r] += a * v[c];
            else        y[c] += a * v[r];
        }
    }
}

/* ------------------------------------ banded LU with partial pivoting (O2) */

/* Working storage: n rows of 3K+1 slots, W(r, c) = lu[r*(3K+1) + (c-r+K)]
 * for c - r in [-K, 2K].  Row interchanges move entries of the current and
 * trailing columns only; multipliers stay where they were computed, so the
 * factorization is A = P_0 L_0 P_1 L_1 ... P_{n-1} L_{n-1} U (elementary
 * lower factors L_j, interchanges P_j of rows j and ipiv[j]).
 * Returns 0, or j+1 if column j has no nonzero pivot candidate. */
#define W3(r, c) lu[(r) * (int64_t)(3 * k + 1) + ((c) - (r) + k)]

int32_t orc_gb_factor(int64_t n, int32_t k, const double *band, double *lu,
                      int64_t *ipiv)
{
    int64_t ldw = 3 * (int64_t)k + 1;
    memset(lu, 0, sizeof(double) * (size_t)(n * ldw));
    for (int64_t r = 0; r < n; ++r) {
        int64_t c0 = r - k < 0 ? 0 : r - k;
        int64_t c1 = r + k > n - 1 ? n - 1 : r + k;
        for (int64_t c = c0; c <= c1; ++c)
            W3(r, c) = band[(int64_t)(k + r - c) * n + c];
    }
    int32_t info = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t last = j + k > n - 1 ? n - 1 : j + k;
        int64_t cend = j + 2 * (int64_t)k > n - 1 ? n - 1 : j + 2 * (int64_t)k;
        int64_t p = j;
        for (int64_t r = j + 1; r <= last; ++r)
            if (fabs(W3(r, j)) > fabs(W3(p, j))) p = r;
        ipiv[j] = p;
        if (W3(p, j) == 0.0) { if (!info) info = (int32_t)(j + 1); continue; }
        if (p != j)
            for (int64_t c = j; c <= cend; ++c) {
                double t = W3(j, c); W3(j, c) = W3(p, c); W3(p, c) = t;
            }
        for (int64_t r = j + 1; r <= last; ++r) {
            double l = W3(r, j) / W3(j, j);
            W3(r, j) = l;
            for (int64_t c = j + 1; c <= cend; ++c) W3(r, c) -= l * W3(j, c);
        }
    }
    return info;
}

/* Solve A x = b (trans = 0) or A^T x = b (trans = 1) in place in x. */
void orc_gb_solve(int64_t n, int32_t k, const double *lu, const int64_t *ipiv,
                  double *x, int32_t trans)
{
    if (!trans) {
        for (int64_t j = 0; j < n; ++j) {                 /* L and P */
            int64_t p = ipiv[j];
            if (p != j) { double t = x[j]; x[j] = x[p]; x[p] = t; }
            int64_t last = j + k > n - 1 ? n - 1 : j + k;
            for (int64_t r = j + 1; r <= last; ++r) x[r] -= W3(r, j) * x[j];
        }
        for (int64_t j = n - 1; j >= 0; --j) {            /* U */
            int64_t cend = j + 2 * (int64_t)k > n - 1 ? n - 1 : j + 2 * (int64_t)k;
            double s = x[j];
            for (int64_t c = j + 1; c <= cend; ++c) s -= W3(j, c) * x[c];
            x[j] = s / W3(j, j);
        }
    } else {
        for (int64_t j = 0; j < n; ++j) {                 /* U^T */
            int64_t i0 = j - 2 * (int64_t)k < 0 ? 0 : j - 2 * (int64_t)k;
            double s = x[j];
            for (int64_t i = i0; i < j; ++i) s -= W3(i, j) * x[i];
            x[j] = s / W3(j, j);
        }
        for (int64_t j = n - 1; j >= 0; --j) {            /* L_j^T then P_j */
            int64_t last = j + k > n - 1 ? n - 1 : j + k;
            double s = x[j];
            for (int64_t r = j + 1; r <= last; ++r) s -= W3(r, j) * x[r];
            x[j] = s;
            int64_t p = ipiv[j];
            if (p != j) { double t = x[j]; x[j] = x[p]; x[p] = t; }
        }
    }
}
#undef W3

/* ------------------------------- block LU / UL without pivoting (SaP) */

#define RW(r, c) f[(r) * (int64_t)(2 * k + 1) + ((c) - (r) + k)]

/* Copy the diagonal block rows/cols [s0, s0+nb) of A into the row window. */
void orc_block_load(int64_t n, int32_t k, const double *band, int64_t s0,
                    int64_t nb, double *f)
{
    memset(f, 0, sizeof(double) * (size_t)(nb * (2 * (int64_t)k + 1)));
    for (int64_t r = 0; r < nb; ++r) {
        int64_t c0 = r - k < 0 ? 0 : r - k;
        int64_t c1 = r + k > nb - 1 ? nb - 1 : r + k;
        for (int64_t c = c0; c <= c1; ++c) {
            int64_t gr = s0 + r, gc = s0 + c;
            RW(r, c) = band[(int64_t)(k + gr - gc) * n + gc];
        }
    }
}

/* Largest |a_rc| over the block (entrywise max norm used for the boost). */
double orc_block_maxabs(int64_t nb, int32_t k, const double *f)
{
    double m = 0.0;
    for (int64_t r = 0; r < nb; ++r) {
        int64_t c0 = r - k < 0 ? 0 : r - k;
        int64_t c1 = r + k > nb - 1 ? nb - 1 : r + k;
        for (int64_t c = c0; c <= c1; ++c)
            if (fabs(RW(r, c)) > m) m = fabs(RW(r, c));
    }
    return m;
}

/* Pivot boosting: a pivot of magnitude below tau becomes +-tau (sign kept,
 * zero taken as positive).  tau < 0 disables boosting. */
static double boost(double p, double tau, int32_t *nboost)
{
    if (tau > 0.0 && fabs(p) < tau) {
        ++*nboost;
        return p >= 0.0 ? tau : -tau;
    }
    return p;
}

/* In-place LU (Doolittle: L unit lower, U upper) of one block, no pivoting.
 * Returns 0, or j+1 if pivot j is exactly zero (possible only with boosting
 * disabled). */
int32_t orc_block_lu(int64_t nb, int32_t k, double *f, double tau, int32_t *nboost)
{
    *nboost = 0;
    for (int64_t j = 0; j < nb; ++j) {
        double p = boost(RW(j, j), tau, nboost);
        RW(j, j) = p;
        if (p == 0.0) return (int32_t)(j + 1);
        int64_t last = j + k > nb - 1 ? nb - 1 : j + k;
        for (int64_t r = j + 1; r <= last; ++r) {
            double l = RW(r, j) / p;
            RW(r, j) = l;
            for (int64_t c = j + 1; c <= last; ++c) RW(r, c) -= l * RW(j, c);
        }
    }
    return 0;
}

/* In-place UL of one block, no pivoting: eliminate from the last row up,
 * giving A = U' L' with U' unit upper (multipliers stored above the
 * diagonal) and L' lower (stored on and below the diagonal). */
int32_t orc_block_ul(int64_t nb, int32_t k, double *f, double tau, int32_t *nboost)
{
    *nboost = 0;
    for (int64_t j = nb - 1; j >= 0; --j) {
        double p = boost(RW(j, j), tau, nboost);
        RW(j, j) = p;
        if (p == 0.0) return (int32_t)(j + 1);
        int64_t first = j - k < 0 ? 0 : j - k;
        for (int64_t r = first; r < j; ++r) {
            double u = RW(r, j) / p;
            RW(r, j) = u;
            for (int64_t c = first; c < j; ++c) RW(r, c) -= u * RW(j, c);
        }
    }
    return 0;
}

/* x <- A_i^{-1} x (trans = 0: forward with L, back with U) or
 * x <- A_i^{-T} x (trans = 1: forward with U^T, back with L^T). */
void orc_block_solve(int64_t nb, int32_t k, const double *f, double *x,
                     int32_t trans)
{
    if (!trans) {
        for (int64_t j = 0; j < nb; ++j) {
            int64_t last = j + k > nb - 1 ? nb - 1 : j + k;
            for (int64_t r = j + 1; r <= last; ++r) x[r] -= RW(r, j) * x[j];
        }
        for (int64_t j = nb - 1; j >= 0; --j) {
            x[j] /= RW(j, j);
            int64_t first = j - k < 0 ? 0 : j - k;
            for (int64_t r = first; r < j; ++r) x[r] -= RW(r, j) * x[j];
        }
    } else {
        for (int64_t j = 0; j < nb; ++j) {
            int64_t first = j - k < 0 ? 0 : j - k;
            double s = x[j];
            for (int64_t i = first; i < j; ++i) s -= RW(i, j) * x[i];
            x[j] = s / RW(j, j);
        }
        for (int64_t j = nb - 1; j >= 0; --j) {
            int64_t last = j + k > nb - 1 ? nb - 1 : j + k;
            double s = x[j];
            for (int64_t r = j + 1; r <= last; ++r) s -= RW(r, j) * x[r];
            x[j] = s;
        }
    }
}
#undef RW
