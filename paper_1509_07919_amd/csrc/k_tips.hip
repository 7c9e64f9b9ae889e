// Coupling blocks, truncated spike tips and the reduced interface matrices of
// the coupled (SaP-C) preconditioner, arXiv:1509.07919 Sec. 2.1:
//
//   B_i     = A[rows: last K of block i,   cols: first K of block i+1]
//   C_{i+1} = A[rows: first K of block i+1, cols: last K of block i]
//   V_i^(b)     = U_bb^{-1} L_bb^{-1} B_i       -- bottom K rows of the right
//                 spike A_i^{-1}[0;0;B_i] (eq:LeftRightSpikes), from the
//                 bottom-right K x K corners of LU(A_i)
//   W_{i+1}^(t) = L'_tt^{-1} U'_tt^{-1} C_{i+1} -- top K rows of the left
//                 spike A_{i+1}^{-1}[C_{i+1};0;0], from the top-left corners of
//                 the UL factorization A_{i+1} = U' L'
//   Rbar_i = I - W_{i+1}^(t) V_i^(b)            -- eq:solveTopBottom
//
// Rbar_i is factored with partial pivoting and inverted once here, so that
// each preconditioner application only needs small matrix-vector products.
//
// One 256-thread workgroup per interface; thread b owns column b of every
// K x K right-hand side (K <= 255).  The K x K operands stay in global memory
// (L2-resident, a few KB to 260 KB per interface); this step is O(P K^3)
// and runs once per factorization.
#include "sap_internal.h"

namespace sap {

__device__ __forceinline__ void block_sync()
{
    __threadfence();
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_tips(TipsArgs<T> a)
{
    const int i = blockIdx.x;                   // interface i: blocks i, i+1
    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int CS = k + 1;
    const int64_t s1 = a.pt.starts[i + 1];      // first row of block i+1
    const int64_t kk = (int64_t)k * k;
    T *B = a.B + i * kk, *C = a.C + i * kk, *V = a.V + i * kk, *W = a.W + i * kk;
    T *R = a.Rbar + i * kk, *RL = a.Rlu + i * kk, *RI = a.Rinv + i * kk;
    int *piv = a.piv + (int64_t)i * k;
    const T *cn = a.corner + (int64_t)(i + 1) * kk;   // UL corner of block i+1
    const int tid = threadIdx.x;

    // B_i (lower triangular incl. diagonal) and C_{i+1} (upper triangular)
    for (int64_t e = tid; e < kk; e += 256) {
        const int r = (int)(e / k), c = (int)(e % k);
        const int64_t br = s1 - k + r, bc = s1 + c;          // B: a[br][bc]
        B[e] = (c <= r) ? (T)a.band[(int64_t)(k + br - bc) * n + bc] : T(0);
        const int64_t cr = s1 + r, cc = s1 - k + c;          // C: a[cr][cc]
        C[e] = (r <= c) ? (T)a.band[(int64_t)(k + cr - cc) * n + cc] : T(0);
    }
    block_sync();

    const int64_t base = s1 - k;                // first row of block i's bottom corner
    const int b = tid;
    if (b < k) {
        // V = U_bb^{-1} (L_bb^{-1} B) on column b.
        // L_bb[r][c] = l(base+r, base+c) = Lc[(base+c)*CS + (r-c)], r > c.
        for (int r = 0; r < k; ++r) {
            T s = B[r * k + b];
            for (int c = 0; c < r; ++c) s = fma(-a.Lc[(base + c) * CS + (r - c)], V[c * k + b], s);
            V[r * k + b] = s;
        }
        // U_bb[r][c] = u(base+r, base+c) = Uc[(base+c)*CS + (c-r)], c > r;
        // 1/u(base+r, base+r) = Uc[(base+r)*CS].
        for (int r = k - 1; r >= 0; --r) {
            T s = V[r * k + b];
            for (int c = r + 1; c < k; ++c) s = fma(-a.Uc[(base + c) * CS + (c - r)], V[c * k + b], s);
            V[r * k + b] = s * a.Uc[(base + r) * CS];
        }
        // W = L'_tt^{-1} (U'_tt^{-1} C).  With the corner cn of LU(J A J):
        // U'_tt[r][c] = cn[(k-1-r)*k + (k-1-c)] for r < c (unit diagonal),
        // L'_tt[r][c] = cn[(k-1-r)*k + (k-1-c)] for r >= c.
        for (int r = k - 1; r >= 0; --r) {
            T s = C[r * k + b];
            for (int c = r + 1; c < k; ++c)
                s = fma(-cn[(k - 1 - r) * k + (k - 1 - c)], W[c * k + b], s);
            W[r * k + b] = s;
        }
        for (int r = 0; r < k; ++r) {
            T s = W[r * k + b];
            for (int c = 0; c < r; ++c)
                s = fma(-cn[(k - 1 - r) * k + (k - 1 - c)], W[c * k + b], s);
            W[r * k + b] = s / cn[(k - 1 - r) * k + (k - 1 - r)];
        }
    }
    block_sync();
    // Rbar = I - W V (column b)
    if (b < k) {
        for (int r = 0; r < k; ++r) {
            T s = (r == b) ? T(1) : T(0);
            for (int c = 0; c < k; ++c) s = fma(-W[r * k + c], V[c * k + b], s);
            R[r * k + b] = s;
            RL[r * k + b] = s;
        }
    }
    block_sync();
    // LU with partial pivoting of Rbar (in RL), ties to the lowest row
    __shared__ int pr_sh;
    for (int j = 0; j < k; ++j) {
        if (tid == 0) {
            int p = j;
            T best = fabs(RL[j * k + j]);
            for (int r = j + 1; r < k; ++r) {
                const T v = fabs(RL[r * k + j]);
                if (v > best) { best = v; p = r; }
            }
            piv[j] = p;
            pr_sh = p;
            if (best == T(0)) a.status[1] = 2;
        }
        block_sync();
        const int p = pr_sh;
        if (p != j)
            for (int c = tid; c < k; c += 256) {
                const T t = RL[j * k + c];
                RL[j * k + c] = RL[p * k + c];
                RL[p * k + c] = t;
            }
        block_sync();
        const T d = RL[j * k + j];
        for (int r = j + 1 + tid; r < k; r += 256) RL[r * k + j] = RL[r * k + j] / d;
        block_sync();
        for (int c = j + 1 + tid; c < k; c += 256) {
            const T ujc = RL[j * k + c];
            for (int r = j + 1; r < k; ++r) RL[r * k + c] = fma(-RL[r * k + j], ujc, RL[r * k + c]);
        }
        block_sync();
    }
    // Rinv = Rbar^{-1}: column b solves Rbar x = e_b with the pivoted LU
    if (b < k) {
        for (int r = 0; r < k; ++r) RI[r * k + b] = (r == b) ? T(1) : T(0);
        for (int j = 0; j < k; ++j) {                  // apply interchanges
            const int p = piv[j];
            if (p != j) {
                const T t = RI[j * k + b];
                RI[j * k + b] = RI[p * k + b];
                RI[p * k + b] = t;
            }
        }
        for (int r = 0; r < k; ++r) {                  // unit lower
            T s = RI[r * k + b];
            for (int c = 0; c < r; ++c) s = fma(-RL[r * k + c], RI[c * k + b], s);
            RI[r * k + b] = s;
        }
        for (int r = k - 1; r >= 0; --r) {            // upper
            T s = RI[r * k + b];
            for (int c = r + 1; c < k; ++c) s = fma(-RL[r * k + c], RI[c * k + b], s);
            RI[r * k + b] = s / RL[r * k + r];
        }
    }
}

template <typename T>
hipError_t launch_tips(const TipsArgs<T> &a, hipStream_t s)
{
    if (a.pt.p < 2) return hipSuccess;
    hipLaunchKernelGGL(k_tips<T>, dim3(a.pt.p - 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_tips<float>(const TipsArgs<float> &, hipStream_t);
template hipError_t launch_tips<double>(const TipsArgs<double> &, hipStream_t);

}  // namespace sap
