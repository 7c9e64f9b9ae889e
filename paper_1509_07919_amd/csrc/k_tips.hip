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
// K x K right-hand side (K <= 255).  The two K x K working matrices live in
// LDS when they fit (2 K^2 elements <= 96 KB), else in global memory; the
// factor corners are read from global memory (L1/L2 resident).  This step is
// O(P K^3) and runs once per factorization.
#include "sap_internal.h"

namespace sap {

// Workgroup barrier that also orders the workgroup's global-memory
// accesses (needed only when the working matrices live in global memory).
template <bool LDS>
__device__ __forceinline__ void block_sync()
{
    if (!LDS) __threadfence_block();
    __syncthreads();
}

// X and Y are the two K x K working matrices (row-major, thread b owns
// column b): in LDS when 2*K*K elements fit, else in the Rlu / Rinv slots of
// global memory.
template <typename T, bool LDS>
__global__ __launch_bounds__(256) void k_tips(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;                   // interface i: blocks i, i+1
    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int CS = k + 1;
    const int64_t s1 = a.pt.starts[i + 1];      // first row of block i+1
    const int64_t kk = (int64_t)k * k;
    T *B = a.B + i * kk, *C = a.C + i * kk, *V = a.V + i * kk, *W = a.W + i * kk;
    T *R = a.Rbar + i * kk, *RI = a.Rinv + i * kk;
    T *X = LDS ? reinterpret_cast<T *>(smem_raw) : a.Rlu + i * kk;
    T *Y = LDS ? reinterpret_cast<T *>(smem_raw) + kk : RI;
    int *piv = a.piv + (int64_t)i * k;
    const T *cn = a.corner + (int64_t)(i + 1) * kk;   // UL corner of block i+1
    const int tid = threadIdx.x;
    __shared__ int pr_sh;

    // B_i (lower triangular incl. diagonal) and C_{i+1} (upper triangular)
    for (int64_t e = tid; e < kk; e += 256) {
        const int r = (int)(e / k), c = (int)(e % k);
        const int64_t br = s1 - k + r, bc = s1 + c;          // B: a[br][bc]
        B[e] = (c <= r) ? (T)a.band[(int64_t)(k + br - bc) * n + bc] : T(0);
        const int64_t cr = s1 + r, cc = s1 - k + c;          // C: a[cr][cc]
        C[e] = (r <= c) ? (T)a.band[(int64_t)(k + cr - cc) * n + cc] : T(0);
    }
    block_sync<LDS>();

    const int64_t base = s1 - k;                // first row of block i's bottom corner
    const int b = tid;
    if (b < k) {
        // V = U_bb^{-1} (L_bb^{-1} B) on column b, working column in X.
        // L_bb[r][c] = l(base+r, base+c) = Lc[(base+c)*CS + (r-c)], r > c.
        for (int r = 0; r < k; ++r) {
            T s = B[r * k + b];
            for (int c = 0; c < r; ++c) s = fma(-a.Lc[(base + c) * CS + (r - c)], X[c * k + b], s);
            X[r * k + b] = s;
        }
        // U_bb[r][c] = u(base+r, base+c) = Uc[(base+c)*CS + (c-r)], c > r;
        // 1/u(base+r, base+r) = Uc[(base+r)*CS].
        for (int r = k - 1; r >= 0; --r) {
            T s = X[r * k + b];
            for (int c = r + 1; c < k; ++c) s = fma(-a.Uc[(base + c) * CS + (c - r)], X[c * k + b], s);
            X[r * k + b] = s * a.Uc[(base + r) * CS];
        }
        for (int r = 0; r < k; ++r) V[r * k + b] = X[r * k + b];
        // W = L'_tt^{-1} (U'_tt^{-1} C) on column b, working column in Y.
        // With the corner cn of LU(J A J): U'_tt[r][c] = cn[(k-1-r)*k + (k-1-c)]
        // for r < c (unit diagonal), L'_tt[r][c] = cn[(k-1-r)*k + (k-1-c)], r >= c.
        for (int r = k - 1; r >= 0; --r) {
            T s = C[r * k + b];
            for (int c = r + 1; c < k; ++c)
                s = fma(-cn[(k - 1 - r) * k + (k - 1 - c)], Y[c * k + b], s);
            Y[r * k + b] = s;
        }
        for (int r = 0; r < k; ++r) {
            T s = Y[r * k + b];
            for (int c = 0; c < r; ++c)
                s = fma(-cn[(k - 1 - r) * k + (k - 1 - c)], Y[c * k + b], s);
            Y[r * k + b] = s / cn[(k - 1 - r) * k + (k - 1 - r)];
        }
        for (int r = 0; r < k; ++r) W[r * k + b] = Y[r * k + b];
    }
    block_sync<LDS>();
    // Rbar = I - W V (column b), from the working copies; Rbar kept in X
    if (b < k) {
        for (int r = 0; r < k; ++r) {
            T s = (r == b) ? T(1) : T(0);
            for (int c = 0; c < k; ++c) s = fma(-Y[r * k + c], X[c * k + b], s);
            R[r * k + b] = s;
        }
    }
    block_sync<LDS>();
    for (int64_t e = tid; e < kk; e += 256) X[e] = R[e];
    block_sync<LDS>();
    // LU with partial pivoting of Rbar in X, ties to the lowest row
    for (int j = 0; j < k; ++j) {
        if (tid == 0) {
            int p = j;
            T best = fabs(X[j * k + j]);
            for (int r = j + 1; r < k; ++r) {
                const T v = fabs(X[r * k + j]);
                if (v > best) { best = v; p = r; }
            }
            piv[j] = p;
            pr_sh = p;
            if (best == T(0)) a.status[1] = 2;
        }
        block_sync<LDS>();
        const int p = pr_sh;
        if (p != j)
            for (int c = tid; c < k; c += 256) {
                const T t = X[j * k + c];
                X[j * k + c] = X[p * k + c];
                X[p * k + c] = t;
            }
        block_sync<LDS>();
        const T d = X[j * k + j];
        for (int r = j + 1 + tid; r < k; r += 256) X[r * k + j] = X[r * k + j] / d;
        block_sync<LDS>();
        for (int c = j + 1 + tid; c < k; c += 256) {
            const T ujc = X[j * k + c];
            for (int r = j + 1; r < k; ++r) X[r * k + c] = fma(-X[r * k + j], ujc, X[r * k + c]);
        }
        block_sync<LDS>();
    }
    // Rinv = Rbar^{-1}: column b solves Rbar y = e_b with the pivoted LU (in Y)
    if (b < k) {
        for (int r = 0; r < k; ++r) Y[r * k + b] = (r == b) ? T(1) : T(0);
        for (int j = 0; j < k; ++j) {                  // apply interchanges
            const int p = piv[j];
            if (p != j) {
                const T t = Y[j * k + b];
                Y[j * k + b] = Y[p * k + b];
                Y[p * k + b] = t;
            }
        }
        for (int r = 0; r < k; ++r) {                  // unit lower
            T s = Y[r * k + b];
            for (int c = 0; c < r; ++c) s = fma(-X[r * k + c], Y[c * k + b], s);
            Y[r * k + b] = s;
        }
        for (int r = k - 1; r >= 0; --r) {            // upper
            T s = Y[r * k + b];
            for (int c = r + 1; c < k; ++c) s = fma(-X[r * k + c], Y[c * k + b], s);
            Y[r * k + b] = s / X[r * k + r];
        }
        if (LDS)
            for (int r = 0; r < k; ++r) RI[r * k + b] = Y[r * k + b];
    }
}

template <typename T>
hipError_t launch_tips(const TipsArgs<T> &a, hipStream_t s)
{
    if (a.pt.p < 2) return hipSuccess;
    const size_t lds = 2 * (size_t)a.pt.k * a.pt.k * sizeof(T);
    if (lds <= 96 * 1024) {
        auto kern = k_tips<T, true>;
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(a.pt.p - 1), dim3(256), lds, s, a);
    } else {
        hipLaunchKernelGGL((k_tips<T, false>), dim3(a.pt.p - 1), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template hipError_t launch_tips<float>(const TipsArgs<float> &, hipStream_t);
template hipError_t launch_tips<double>(const TipsArgs<double> &, hipStream_t);

}  // namespace sap
