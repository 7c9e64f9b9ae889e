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
// K x K right-hand side (K <= 255).  The working matrices and both staged
// factor corners live in LDS when they fit (4 K^2 elements <= 128 KB); then
// the V and W solves run side by side (threads 0..K-1 and K..2K-1).  Else
// they live in global memory and the two solves run one after the other.
// This step is O(P K^3) and runs once per factorization.
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

// dot of row r of M (entries c in [c0, c1)) with column b of X, both row-major
// K x K in the same memory space; four partial sums shorten the FMA chain
template <typename T>
__device__ __forceinline__ T rowdot(const T *M, const T *X, int k, int r, int b, int c0, int c1)
{
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int c = c0;
    for (; c + 3 < c1; c += 4) {
        s0 = fma(M[r * k + c], X[c * k + b], s0);
        s1 = fma(M[r * k + c + 1], X[(c + 1) * k + b], s1);
        s2 = fma(M[r * k + c + 2], X[(c + 2) * k + b], s2);
        s3 = fma(M[r * k + c + 3], X[(c + 3) * k + b], s3);
    }
    for (; c < c1; ++c) s0 = fma(M[r * k + c], X[c * k + b], s0);
    return (s0 + s1) + (s2 + s3);
}

// X, Y (right-hand-side columns, thread b owns column b) and F (the staged
// K x K factor corner, later Rbar and its LU) are row-major K x K working
// matrices, with G (the second corner) in LDS mode: in LDS when 4*K*K
// elements fit, else in global memory (the V, W and Rlu slots; the Rinv
// columns are then solved in place in Rinv).
template <typename T, bool LDS>
__global__ __launch_bounds__(256) void k_tips(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;                   // interface i: blocks i, i+1
    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int CS = k + 1;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int64_t s1 = a.pt.starts[i + 1];      // first row of block i+1
    const int64_t kk = (int64_t)k * k;
    T *B = a.B + i * kk, *C = a.C + i * kk, *V = a.V + i * kk, *W = a.W + i * kk;
    T *R = a.Rbar + i * kk, *RI = a.Rinv + i * kk;
    T *X = LDS ? reinterpret_cast<T *>(smem_raw) : V;
    T *Y = LDS ? reinterpret_cast<T *>(smem_raw) + kk : W;
    T *F = LDS ? reinterpret_cast<T *>(smem_raw) + 2 * kk : a.Rlu + i * kk;
    T *Z = LDS ? Y : RI;                        // Rinv working columns
    int *piv = a.piv + (int64_t)i * k;
    const T *cn = a.corner + (int64_t)(i + 1) * kk;   // UL corner of block i+1
    const int tid = threadIdx.x;
    const int64_t base = s1 - k;                // first row of block i's bottom corner
    __shared__ int pr_sh;
    __shared__ int piv_sh[kMaxK];
    __shared__ T zero_sh;

    // B_i (lower triangular incl. diagonal) -> X, C_{i+1} (upper triangular)
    // -> Y, and the bottom-right corner of LU(A_i) -> F, with
    // F[r][c] = l(base+r, base+c) for r > c (unit diagonal implied) and
    // F[r][c] = u(base+r, base+c) for r <= c; the stored diagonal of U is
    // its reciprocal.  In LDS mode the reversed corner of LU(J A_{i+1} J) goes
    // to G at the same time: U'_tt (unit upper) above the diagonal, L'_tt on
    // and below it.
    T *G = LDS ? reinterpret_cast<T *>(smem_raw) + 3 * kk : nullptr;
    for (int64_t e = tid; e < kk; e += 256) {
        const int r = (int)(e / k), c = (int)(e % k);
        const int64_t br = s1 - k + r, bc = s1 + c;          // B: a[br][bc]
        const T bv = (c <= r) ? (T)a.band[(int64_t)(k + br - bc) * n + bc] : T(0);
        const int64_t cr = s1 + r, cc = s1 - k + c;          // C: a[cr][cc]
        const T cv = (r <= c) ? (T)a.band[(int64_t)(k + cr - cc) * n + cc] : T(0);
        B[e] = bv;
        C[e] = cv;
        X[e] = bv;
        Y[e] = cv;
        F[e] = (r > c) ? a.Lc[(base + c) * CP + (r - c)]
                       : a.Uc[(base + c) * CP + (c - r)];    // c == r: 1/u_rr
        if (LDS) G[e] = cn[(int64_t)(k - 1 - r) * k + (k - 1 - c)];
    }
    if (tid == 0) zero_sh = T(0);
    block_sync<LDS>();

    const int b = tid;
    if (LDS) {
        // V (threads 0..K-1) and W (threads K..2K-1) at the same time
        if (b < k) {
            // V = U_bb^{-1} (L_bb^{-1} B_i), column b, in X
            for (int r = 1; r < k; ++r) X[r * k + b] -= rowdot(F, X, k, r, b, 0, r);
            for (int r = k - 1; r >= 0; --r)
                X[r * k + b] = (X[r * k + b] - rowdot(F, X, k, r, b, r + 1, k)) * F[r * k + r];
        } else if (b < 2 * k) {
            // W = L'_tt^{-1} (U'_tt^{-1} C_{i+1}), column b - K, in Y
            const int w = b - k;
            for (int r = k - 2; r >= 0; --r) Y[r * k + w] -= rowdot(G, Y, k, r, w, r + 1, k);
            for (int r = 0; r < k; ++r)
                Y[r * k + w] = (Y[r * k + w] - rowdot(G, Y, k, r, w, 0, r)) / G[r * k + r];
        }
        block_sync<LDS>();
        for (int64_t e = tid; e < kk; e += 256) V[e] = X[e];
    } else {
        if (b < k) {
            // V = U_bb^{-1} (L_bb^{-1} B_i), column b, in X
            for (int r = 1; r < k; ++r) X[r * k + b] -= rowdot(F, X, k, r, b, 0, r);
            for (int r = k - 1; r >= 0; --r)
                X[r * k + b] = (X[r * k + b] - rowdot(F, X, k, r, b, r + 1, k)) * F[r * k + r];
        }
        block_sync<LDS>();
        // corner of LU(J A_{i+1} J) -> F reversed: F[r][c] = cn[(k-1-r)*k + (k-1-c)],
        // i.e. U'_tt (unit upper) above the diagonal and L'_tt on and below it
        for (int64_t e = tid; e < kk; e += 256) {
            const int r = (int)(e / k), c = (int)(e % k);
            F[e] = cn[(int64_t)(k - 1 - r) * k + (k - 1 - c)];
            V[e] = X[e];
        }
        block_sync<LDS>();
        if (b < k) {
            // W = L'_tt^{-1} (U'_tt^{-1} C_{i+1}), column b, in Y
            for (int r = k - 2; r >= 0; --r) Y[r * k + b] -= rowdot(F, Y, k, r, b, r + 1, k);
            for (int r = 0; r < k; ++r)
                Y[r * k + b] = (Y[r * k + b] - rowdot(F, Y, k, r, b, 0, r)) / F[r * k + r];
        }
    }
    block_sync<LDS>();
    // Rbar = I - W V -> F and R (global)
    for (int64_t e = tid; e < kk; e += 256) W[e] = Y[e];
    if (b < k) {
        for (int r = 0; r < k; ++r) {
            const T s = ((r == b) ? T(1) : T(0)) - rowdot(Y, X, k, r, b, 0, k);
            R[r * k + b] = s;
            F[r * k + b] = s;
        }
    }
    block_sync<LDS>();
    // LU with partial pivoting of Rbar in F (ties to the lowest row); the
    // pivot search is a wave-0 argmax
    for (int j = 0; j < k; ++j) {
        if (tid < 64) {
            T best = T(-1);
            int p = j;
            for (int r = j + tid; r < k; r += 64) {
                const T v = fabs(F[r * k + j]);
                if (v > best) { best = v; p = r; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const T ob = __shfl_xor(best, o, 64);
                const int op = __shfl_xor(p, o, 64);
                if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
            }
            if (tid == 0) {
                piv[j] = p;
                piv_sh[j] = p;
                pr_sh = p;
                if (best == T(0)) a.status[1] = 2;
            }
        }
        block_sync<LDS>();
        const int p = pr_sh;
        if (p != j)
            for (int c = tid; c < k; c += 256) {
                const T t = F[j * k + c];
                F[j * k + c] = F[p * k + c];
                F[p * k + c] = t;
            }
        block_sync<LDS>();
        const T d = F[j * k + j];
        const T dinv = d != T(0) ? T(1) / d : zero_sh;
        const int m = k - 1 - j;                               // trailing size
        for (int e = tid; e < m * m; e += 256) {
            const int r = j + 1 + e / m, c = j + 1 + e % m;
            F[r * k + c] = fma(-F[r * k + j] * dinv, F[j * k + c], F[r * k + c]);
        }
        block_sync<LDS>();
        for (int r = j + 1 + tid; r < k; r += 256) F[r * k + j] *= dinv;
        block_sync<LDS>();
    }
    // Rinv = Rbar^{-1}: column b solves Rbar y = e_b with the pivoted LU (in Z)
    if (b < k) {
        for (int r = 0; r < k; ++r) Z[r * k + b] = (r == b) ? T(1) : T(0);
        for (int j = 0; j < k; ++j) {                  // apply interchanges
            const int p = piv_sh[j];
            if (p != j) {
                const T t = Z[j * k + b];
                Z[j * k + b] = Z[p * k + b];
                Z[p * k + b] = t;
            }
        }
        for (int r = 1; r < k; ++r) Z[r * k + b] -= rowdot(F, Z, k, r, b, 0, r);
        for (int r = k - 1; r >= 0; --r)
            Z[r * k + b] = (Z[r * k + b] - rowdot(F, Z, k, r, b, r + 1, k)) / F[r * k + r];
        if (LDS)
            for (int r = 0; r < k; ++r) RI[r * k + b] = Z[r * k + b];
    }
}

template <typename T>
hipError_t launch_tips(const TipsArgs<T> &a, hipStream_t s)
{
    if (a.pt.p < 2) return hipSuccess;
    const size_t lds = 4 * (size_t)a.pt.k * a.pt.k * sizeof(T);
    if (lds <= 128 * 1024 && 2 * a.pt.k <= 256) {
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
