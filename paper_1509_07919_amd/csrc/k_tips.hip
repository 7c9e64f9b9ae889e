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
// Rbar_i is inverted once here (with partial pivoting), so that each
// preconditioner application only needs small matrix-vector products.
//
// One 256-thread workgroup per interface.  When the four K x K working
// matrices fit in LDS, k_tips_lds spreads every step over all threads (K <=
// 71 for FP64 factors, K <= 100 for FP32); else the k_tips_global_* kernels
// keep them in global memory with one thread per right-hand-side column, V
// and W side by side and Rbar split by rows.  This step is O(P K^3) and runs
// once per factorization.
#include "sap_internal.h"

namespace sap {

// Workgroup barrier that also orders the workgroup's global-memory accesses
// (the working matrices of the k_tips_global_* kernels live in global memory).
__device__ __forceinline__ void block_sync()
{
    __threadfence_block();
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

// Global-memory version, for K too large for LDS, in five launches (the
// K x K working matrices are row-major in global memory):
//   k_tips_global_stage grid (P-1, 2): y = 0 stages B_i (into the B and V
//                       slots) and the bottom-right corner of LU(A_i) (into
//                       the Rlu slot); y = 1 stages C_{i+1} (into the C and W
//                       slots) and the corner of the UL factorization (into
//                       the Rbar slot);
//   k_tips_global_vw    grid (P-1, 2 x column groups), one wave: V (y <
//                       groups) or W by substitution, one thread per
//                       right-hand-side column, the wave's 64 columns held in
//                       LDS and the factor corner read from global memory
//                       (the same address in every lane);
//   k_tips_global_rbar  grid (P-1, tiles^2): Rbar = I - W V in 64 x 64
//                       tiles staged through LDS, into the Rbar and Rlu slots;
//   k_tips_global_lu    grid (P-1), 1024 threads: the pivoted LU of Rbar, in LDS when K^2
//                       elements fit (FP32 K <= 202, FP64 K <= 143), stored
//                       in the Rlu slot;
//   k_tips_global_rinv  grid (P-1, column groups), one wave: the Rinv columns
//                       from the pivoted LU, held in LDS like V and W.
// Each column's substitution is a chain over K rows; with the column and the
// factor row in LDS a row waits on LDS only, not on a global round trip.
template <typename T>
__global__ __launch_bounds__(256) void k_tips_global_stage(TipsArgs<T> a)
{
    const int i = blockIdx.x;                   // interface i: blocks i, i+1
    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int64_t s1 = a.pt.starts[i + 1];      // first row of block i+1
    const int64_t kk = (int64_t)k * k;
    const int tid = threadIdx.x;
    if (blockIdx.y == 0) {
        T *B = a.B + i * kk, *X = a.V + i * kk, *F = a.Rlu + i * kk;
        const int64_t base = s1 - k;            // first row of block i's bottom corner
        // B_i (lower triangular incl. diagonal) -> B and X, and the
        // bottom-right corner of LU(A_i) -> F, with F[r][c] = l(base+r,
        // base+c) for r > c (unit diagonal implied) and F[r][c] = u(base+r,
        // base+c) for r <= c; the stored diagonal of U is its reciprocal
        for (int64_t e = tid; e < kk; e += 256) {
            const int r = (int)(e / k), c = (int)(e % k);
            const int64_t br = s1 - k + r, bc = s1 + c;      // B: a[br][bc]
            const T bv = (c <= r) ? (T)a.band[(int64_t)(k + br - bc) * n + bc] : T(0);
            B[e] = bv;
            X[e] = bv;
            F[e] = (r > c) ? a.Lc[(base + c) * CP + (r - c)]
                           : a.Uc[(base + c) * CP + (c - r)];    // c == r: 1/u_rr
        }
    } else {
        T *C = a.C + i * kk, *Y = a.W + i * kk, *F = a.Rbar + i * kk;
        const T *cn = a.corner + (int64_t)(i + 1) * kk;   // UL corner of block i+1
        // C_{i+1} (upper triangular) -> C and Y, and the corner of
        // LU(J A_{i+1} J) reversed -> F: F[r][c] = cn[(k-1-r)*k + (k-1-c)],
        // i.e. U'_tt (unit upper) above the diagonal and L'_tt on and below it
        for (int64_t e = tid; e < kk; e += 256) {
            const int r = (int)(e / k), c = (int)(e % k);
            const int64_t cr = s1 + r, cc = s1 - k + c;      // C: a[cr][cc]
            const T cv = (r <= c) ? (T)a.band[(int64_t)(k + cr - cc) * n + cc] : T(0);
            C[e] = cv;
            Y[e] = cv;
            F[e] = cn[(int64_t)(k - 1 - r) * k + (k - 1 - c)];
        }
    }
}

// Row-by-row substitution on the columns held in LDS (xs[c * 64 + t]) by a
// one-wave workgroup.  FWD: rows rfirst..K-1, each minus its dot over
// columns [0, r); else rows rfirst..0, each minus its dot over [r+1, K).
// DIAG: 0 unit diagonal, 1 multiply by M[r][r] (a stored reciprocal), 2
// divide by it.  The wave stages each factor row in LDS (fs, two K-element
// slots), loading the row after next into registers while it works on the
// current one, so a row waits on LDS only; the dot keeps rowdot's order.
template <typename T, bool FWD, int DIAG>
__device__ __forceinline__ void subst_rows(const T *__restrict__ M, T *xs, T *fs, int k, int t,
                                           int rfirst)
{
    const int nrow = FWD ? k - rfirst : rfirst + 1;
    if (nrow <= 0) return;
    T pre[4];                                   // K <= 255: four entries per lane
    auto issue = [&](int s2) {
        const int r = FWD ? rfirst + s2 : rfirst - s2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = t + 64 * q;
            pre[q] = (s2 < nrow && c < k) ? M[r * k + c] : T(0);
        }
    };
    auto commit = [&](T *dst) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = t + 64 * q;
            if (c < k) dst[c] = pre[q];
        }
        __builtin_amdgcn_wave_barrier();
    };
    issue(0);
    commit(fs);
    issue(1);
    for (int s2 = 0; s2 < nrow; ++s2) {
        const int r = FWD ? rfirst + s2 : rfirst - s2;
        const T *f = fs + (s2 & 1) * k;
        const int c0 = FWD ? 0 : r + 1, c1 = FWD ? r : k;
        T s0 = T(0), s1 = T(0), s2v = T(0), s3 = T(0);
        int c = c0;
        for (; c + 3 < c1; c += 4) {
            s0 = fma(f[c], xs[c * 64 + t], s0);
            s1 = fma(f[c + 1], xs[(c + 1) * 64 + t], s1);
            s2v = fma(f[c + 2], xs[(c + 2) * 64 + t], s2v);
            s3 = fma(f[c + 3], xs[(c + 3) * 64 + t], s3);
        }
        for (; c < c1; ++c) s0 = fma(f[c], xs[c * 64 + t], s0);
        T v = xs[r * 64 + t] - ((s0 + s1) + (s2v + s3));
        if (DIAG == 1) v *= f[r];
        if (DIAG == 2) v /= f[r];
        xs[r * 64 + t] = v;
        __builtin_amdgcn_wave_barrier();
        commit(fs + ((s2 + 1) & 1) * k);
        issue(s2 + 2);
    }
}

// V = U_bb^{-1} (L_bb^{-1} B_i) or W = L'_tt^{-1} (U'_tt^{-1} C_{i+1}) for
// the 64 columns of this workgroup; each thread works on its own column
// only, so the kernel has no barrier
template <typename T>
__global__ __launch_bounds__(64) void k_tips_global_vw(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);    // [K][64]
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int ncg = (k + 63) / 64;
    const int which = (int)blockIdx.y / ncg;    // 0: V, 1: W
    const int t = threadIdx.x;
    const int b = ((int)blockIdx.y % ncg) * 64 + t;
    const int64_t kk = (int64_t)k * k;
    const bool act = b < k;                     // every lane stages factor rows
    T *fs = xs + (size_t)k * 64;                // [2][K]
    T *X = (which == 0 ? a.V : a.W) + i * kk;
    const T *__restrict__ F = (which == 0 ? a.Rlu : a.Rbar) + i * kk;
    for (int c = 0; c < k; ++c) xs[c * 64 + t] = act ? X[c * k + b] : T(0);
    if (which == 0) {
        subst_rows<T, true, 0>(F, xs, fs, k, t, 1);
        subst_rows<T, false, 1>(F, xs, fs, k, t, k - 1);
    } else {
        subst_rows<T, false, 0>(F, xs, fs, k, t, k - 2);
        subst_rows<T, true, 2>(F, xs, fs, k, t, 0);
    }
    if (act)
        for (int c = 0; c < k; ++c) X[c * k + b] = xs[c * 64 + t];
}

// Rbar = I - W V as 64 x 64 output tiles (grid (P-1, tiles^2)): the tile's
// rows of W and columns of V pass through LDS 16 at a time, and each thread
// accumulates a 4 x 4 block of outputs (rows ty + 16 u, columns tx + 16 v)
template <typename T>
__global__ __launch_bounds__(256) void k_tips_global_rbar(TipsArgs<T> a)
{
    constexpr int TB = 64, KC = 16;
    __shared__ T ysh[TB][KC + 1];               // W[r0 + row][c0 + col]
    __shared__ T xsh[KC][TB + 1];               // V[c0 + row][b0 + col]
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int64_t kk = (int64_t)k * k;
    const T *X = a.V + i * kk, *Y = a.W + i * kk;
    T *R = a.Rbar + i * kk, *F = a.Rlu + i * kk;
    const int nt = (k + TB - 1) / TB;
    const int r0 = ((int)blockIdx.y / nt) * TB, b0 = ((int)blockIdx.y % nt) * TB;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    T acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
    for (int c0 = 0; c0 < k; c0 += KC) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;        // 1024 entries of each tile
            const int yr = e >> 4, yc = e & 15;
            ysh[yr][yc] = (r0 + yr < k && c0 + yc < k) ? Y[(int64_t)(r0 + yr) * k + c0 + yc] : T(0);
            const int xr = e >> 6, xc = e & 63;
            xsh[xr][xc] = (c0 + xr < k && b0 + xc < k) ? X[(int64_t)(c0 + xr) * k + b0 + xc] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T yv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) yv[u] = ysh[ty + 16 * u][c];
#pragma unroll
            for (int v = 0; v < 4; ++v) xv[v] = xsh[c][tx + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(yv[u], xv[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = r0 + ty + 16 * u;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int b = b0 + tx + 16 * v;
            if (r < k && b < k) {
                const T s = ((r == b) ? T(1) : T(0)) - acc[u][v];
                R[(int64_t)r * k + b] = s;
                F[(int64_t)r * k + b] = s;
            }
        }
    }
}

// INLDS: Rbar is factored in LDS (K^2 elements of dynamic LDS) and written
// back to the Rlu slot at the end; else in place in the Rlu slot
constexpr int kTipsLuNT = 1024;     // threads of k_tips_global_lu: a 32 x 32 grid

template <typename T, bool INLDS>
__global__ __launch_bounds__(kTipsLuNT) void k_tips_global_lu(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int64_t kk = (int64_t)k * k;
    T *G = a.Rlu + i * kk;
    T *F = INLDS ? reinterpret_cast<T *>(smem_raw) : G;
    int *piv = a.piv + (int64_t)i * k;
    const int tid = threadIdx.x;
    __shared__ int pr_sh;
    __shared__ T zero_sh;
    if (INLDS)
        for (int e = tid; e < kk; e += kTipsLuNT) F[e] = G[e];
    if (tid == 0) zero_sh = T(0);
    block_sync();
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
                pr_sh = p;
                if (best == T(0)) a.status[1] = 2;
            }
        }
        block_sync();
        const int p = pr_sh;
        if (p != j)
            for (int c = tid; c < k; c += kTipsLuNT) {
                const T t = F[j * k + c];
                F[j * k + c] = F[p * k + c];
                F[p * k + c] = t;
            }
        block_sync();
        const T d = F[j * k + j];
        const T dinv = d != T(0) ? T(1) / d : zero_sh;
        // trailing update: thread (tid / 32, tid % 32) takes every 32nd row
        // and column, so no index needs a division
        for (int r = j + 1 + (tid >> 5); r < k; r += 32) {
            const T l = F[r * k + j] * dinv;
            for (int c = j + 1 + (tid & 31); c < k; c += 32)
                F[r * k + c] = fma(-l, F[j * k + c], F[r * k + c]);
        }
        block_sync();
        for (int r = j + 1 + tid; r < k; r += kTipsLuNT) F[r * k + j] *= dinv;
        block_sync();
    }
    if (INLDS)
        for (int e = tid; e < kk; e += kTipsLuNT) G[e] = F[e];
}

// Rinv = Rbar^{-1}: column b solves Rbar y = e_b with the pivoted LU of the
// Rlu slot, held in LDS like V and W
template <typename T>
__global__ __launch_bounds__(64) void k_tips_global_rinv(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);    // [K][64]
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int t = threadIdx.x;
    const int b = (int)blockIdx.y * 64 + t;
    const int64_t kk = (int64_t)k * k;
    const bool act = b < k;                     // every lane stages factor rows
    T *fs = xs + (size_t)k * 64;                // [2][K]
    const T *__restrict__ F = a.Rlu + i * kk;
    const int *__restrict__ piv = a.piv + (int64_t)i * k;
    for (int r = 0; r < k; ++r) xs[r * 64 + t] = (r == b) ? T(1) : T(0);
    for (int j = 0; j < k; ++j) {                      // apply interchanges
        const int p = piv[j];
        if (p != j) {
            const T v = xs[j * 64 + t];
            xs[j * 64 + t] = xs[p * 64 + t];
            xs[p * 64 + t] = v;
        }
    }
    subst_rows<T, true, 0>(F, xs, fs, k, t, 1);
    subst_rows<T, false, 2>(F, xs, fs, k, t, k - 1);
    T *Z = a.Rinv + i * kk;
    if (act)
        for (int r = 0; r < k; ++r) Z[r * k + b] = xs[r * 64 + t];
}


// ---------------------------------------------------------------------------
// The same quantities with every K x K working matrix in LDS (4 K^2 + 3 K
// elements), spread over all NT threads (512, or 1024 for K >= 64, where no
// transfer-matrix kernel runs beside this one):
//   (a) B, C, the two factor corners and 1/diag(L'_tt) are loaded, all loads
//       of a batch issued before the first store;
//   (b) V and W by right-looking (column-sweep) substitution, one pivot row
//       per step and one barrier per step: the first half of the threads
//       works on V, the second on W, element (row, column) pairs spread over
//       the team.  The
//       scaling by a pivot of the non-unit triangle is applied on the fly to
//       the pivot row that the step reads, and written back one step later,
//       when no thread reads that row any more;
//   (c) Rbar = I - W V, one 2 x 4 block of outputs per thread and pass;
//   (d) Rinv by Gauss-Jordan elimination with partial pivoting (ties to the
//       lowest row), in place, three barriers per pivot: wave 0 finds the
//       pivot, all threads stage the scaled pivot row and the pivot column,
//       then every other row is eliminated (the item of the pivot's row also
//       moves the displaced row); the column order is restored when Rinv is
//       written out.
// NT threads: two teams of NT / 2 >= K threads
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_tips_lds(TipsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;                   // interface i: blocks i, i+1
    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int64_t s1 = a.pt.starts[i + 1];      // first row of block i+1
    const int kk = k * k;
    T *X = reinterpret_cast<T *>(smem_raw);     // V
    T *Y = X + kk;                              // W
    T *F = Y + kk;                              // LU corner of block i, then Rbar
    T *G = F + kk;                              // UL corner of block i+1
    T *gi = G + kk;                             // 1 / diag(L'_tt)
    T *colj = gi + k;                           // Gauss-Jordan pivot column
    T *rowj = colj + k;                         // Gauss-Jordan scaled pivot row
    __shared__ int perm_sh[kMaxK], ord_sh[kMaxK];
    __shared__ int p_sh;
    __shared__ T d_sh;
    const int tid = threadIdx.x;
    const int64_t base = s1 - k;                // first row of block i's bottom corner
    // time this workgroup spends in (a) B/C gather (T_BC), (b) spikes
    // (T_SPK) and (c, d) Rbar and its inverse (T_LUrdcd), summed over the
    // workgroups with the constant 100 MHz clock (wall_clock64)
    unsigned long long tk = (a.ticks && tid == 0) ? wall_clock64() : 0ull;
    auto lap = [&](int ph) {
        if (a.ticks && tid == 0) {
            const unsigned long long u = wall_clock64();
            atomicAdd(a.ticks + ph, u - tk);
            tk = u;
        }
    };
    const T *cn = a.corner + (int64_t)(i + 1) * kk;
    const int64_t ikk = (int64_t)i * kk;

    // (a) B_i (lower triangular incl. diagonal) -> X, C_{i+1} (upper
    // triangular) -> Y, the bottom-right corner of LU(A_i) -> F (l below the
    // diagonal, u on and above it with the reciprocal on the diagonal), the
    // reversed corner of LU(J A_{i+1} J) -> G (U'_tt above the diagonal, L'_tt
    // on and below it)
    // thread (gc, gr0) covers column gc, rows gr0 + grs * q (grs = floor(NT / K))
    const int grs = NT / k;
    const int gc = tid % k, gr0 = tid / k;
    const bool gact = gr0 < grs;
    constexpr int QB = 4;
    for (int rb = 0; rb < k; rb += grs * QB) {
        double bv[QB], cv[QB];
        T fv[QB], gv[QB];
        const int c = gc;
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int r = rb + gr0 + grs * q;
            bv[q] = cv[q] = 0.0;
            fv[q] = gv[q] = T(0);
            if (gact && r < k) {
                if (c <= r) bv[q] = a.band[(int64_t)(r - c) * n + s1 + c];
                if (r <= c) cv[q] = a.band[(int64_t)(2 * k + r - c) * n + s1 - k + c];
                fv[q] = (r > c) ? a.Lc[(base + c) * CP + (r - c)] : a.Uc[(base + c) * CP + (c - r)];
                gv[q] = cn[(k - 1 - r) * k + (k - 1 - c)];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int r = rb + gr0 + grs * q;
            if (gact && r < k) {
                const int e = r * k + c;
                a.B[ikk + e] = (T)bv[q];
                a.C[ikk + e] = (T)cv[q];
                X[e] = (T)bv[q];
                Y[e] = (T)cv[q];
                F[e] = fv[q];
                G[e] = gv[q];
            }
        }
    }
    __syncthreads();
    for (int c = tid; c < k; c += NT) gi[c] = T(1) / G[c * k + c];
    __syncthreads();
    lap(0);

    // (b) V = U_bb^{-1} (L_bb^{-1} B_i) in X, W = L'_tt^{-1} (U'_tt^{-1} C_{i+1}) in Y
    // a team thread owns column tc and the rows congruent to tr0 modulo
    // trs = floor(NT / 2 / K) (threads past trs*K idle), so no step divides
    const bool vteam = tid < NT / 2;
    const int tt = vteam ? tid : tid - NT / 2;
    const int trs = NT / 2 / k;
    const int tc = tt % k, tr0 = tt / k;
    const bool tact = tr0 < trs;
    // unit triangles: V forward with L_bb (step s: pivot row s), W backward
    // with U'_tt (pivot row k-1-s)
    for (int s = 0; s + 1 < k; ++s) {
        if (tact) {
            if (vteam) {
                const int c = s;
                const T xc = X[c * k + tc];
                for (int r = c + 1 + tr0; r < k; r += trs)
                    X[r * k + tc] = fma(-F[r * k + c], xc, X[r * k + tc]);
            } else {
                const int c = k - 1 - s;
                const T yc = Y[c * k + tc];
                for (int r = tr0; r < c; r += trs)
                    Y[r * k + tc] = fma(-G[r * k + c], yc, Y[r * k + tc]);
            }
        }
        __syncthreads();
    }
    // non-unit triangles: V backward with U_bb (pivot row k-1-s, scaled by
    // the stored reciprocal), W forward with L'_tt (pivot row s, scaled by gi)
    for (int s = 0; s < k; ++s) {
        if (tact) {
            if (vteam) {
                const int c = k - 1 - s;
                const T xc = X[c * k + tc] * F[c * k + c];
                for (int r = tr0; r < c; r += trs)
                    X[r * k + tc] = fma(-F[r * k + c], xc, X[r * k + tc]);
                if (c + 1 < k && tr0 == 0)      // the previous pivot row
                    X[(c + 1) * k + tc] *= F[(c + 1) * k + c + 1];
            } else {
                const int c = s;
                const T yc = Y[c * k + tc] * gi[c];
                for (int r = c + 1 + tr0; r < k; r += trs)
                    Y[r * k + tc] = fma(-G[r * k + c], yc, Y[r * k + tc]);
                if (c > 0 && tr0 == 0)
                    Y[(c - 1) * k + tc] *= gi[c - 1];
            }
        }
        __syncthreads();
    }
    if (tact && tr0 == 0) {
        if (vteam) X[tc] *= F[0];
        else Y[(k - 1) * k + tc] *= gi[k - 1];
    }
    __syncthreads();
    for (int e = tid; e < kk; e += NT) {
        a.V[ikk + e] = X[e];
        a.W[ikk + e] = Y[e];
    }
    lap(1);

    // (c) Rbar = I - W V -> F and Rbar (global); item (row pair, 4 columns)
    {
        const int ng = (k + 3) / 4, nr = (k + 1) / 2;
        for (int it = tid; it < nr * ng; it += NT) {
            const int r0 = 2 * (it / ng), c0 = 4 * (it - (it / ng) * ng);
            const int r1 = min(r0 + 1, k - 1);
            T acc0[4] = {T(0), T(0), T(0), T(0)}, acc1[4] = {T(0), T(0), T(0), T(0)};
            for (int m = 0; m < k; ++m) {
                const T y0 = Y[r0 * k + m], y1 = Y[r1 * k + m];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T xv = X[m * k + min(c0 + q, k - 1)];
                    acc0[q] = fma(y0, xv, acc0[q]);
                    acc1[q] = fma(y1, xv, acc1[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = c0 + q;
                if (c >= k) continue;
                const T v0 = ((r0 == c) ? T(1) : T(0)) - acc0[q];
                F[r0 * k + c] = v0;
                a.Rbar[ikk + r0 * k + c] = v0;
                if (r0 + 1 < k) {
                    const T v1 = ((r0 + 1 == c) ? T(1) : T(0)) - acc1[q];
                    F[(r0 + 1) * k + c] = v1;
                    a.Rbar[ikk + (r0 + 1) * k + c] = v1;
                }
            }
        }
    }
    __syncthreads();

    // (d) Gauss-Jordan inversion of Rbar in F with row interchanges (thread
    // (gc, gr0) as in (a))
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
                const T pv = F[p * k + j];
                perm_sh[j] = p;
                p_sh = p;
                if (pv == T(0)) a.status[1] = 2;
                d_sh = pv != T(0) ? T(1) / pv : T(0);
            }
        }
        __syncthreads();
        const int p = p_sh;
        const T d = d_sh;
        // staged pivot row (the new row j, scaled) and pivot column (by the
        // row each entry will sit in after the interchange)
        if (tid < k) {
            const int c = tid;
            rowj[c] = (c == j ? T(1) : F[p * k + c]) * d;
        } else if (tid >= NT / 2 && tid - NT / 2 < k) {
            const int r = tid - NT / 2;
            const int src = r == j ? p : (r == p ? j : r);
            colj[r] = F[src * k + j];
        }
        __syncthreads();
        if (gact) {
            const int c = gc;
            const T rc = rowj[c];
            // the row that moves to p (when p != j) is handled with row p
            for (int r = gr0; r < k; r += grs) {
                if (r == j) {
                    if (p == j) F[j * k + c] = rc;
                } else if (r == p) {
                    const T old = c == j ? T(0) : F[j * k + c];
                    F[j * k + c] = rc;
                    F[p * k + c] = fma(-colj[p], rc, old);
                } else {
                    const T old = c == j ? T(0) : F[r * k + c];
                    F[r * k + c] = fma(-colj[r], rc, old);
                }
            }
        }
        __syncthreads();
    }
    // Rinv = F P_{K-1} ... P_0 (P_j swaps j and perm[j]): undoing the
    // interchanges from the last to the first maps output column c to column
    // ord[c] of F
    if (tid == 0) {
        for (int c = 0; c < k; ++c) ord_sh[c] = c;
        for (int j = k - 1; j >= 0; --j) {
            const int q = perm_sh[j];
            const int t = ord_sh[j];
            ord_sh[j] = ord_sh[q];
            ord_sh[q] = t;
        }
    }
    __syncthreads();
    for (int r = gr0; gact && r < k; r += grs) a.Rinv[ikk + r * k + gc] = F[r * k + ord_sh[gc]];
    lap(2);
}

// the four K x K working matrices and 3K vectors in LDS, plus the static LDS
// of k_tips_lds (perm_sh, ord_sh, p_sh, d_sh)
bool tips_in_lds(int k, bool fp32)
{
    const size_t ts = fp32 ? 4 : 8;
    const size_t kk = (size_t)k * k;
    return (4 * kk + 3 * (size_t)k) * ts + 2 * kMaxK * sizeof(int) + sizeof(int) + ts + 64 <= kMaxLds;
}

// ev (nullable): events recorded before the first launch, after the B/C
// gather, after the spikes and after the last launch; in the LDS form the
// middle two are not recorded (its phases are split by a.ticks instead)
template <typename T>
hipError_t launch_tips(const TipsArgs<T> &a, hipStream_t s, hipEvent_t *ev)
{
    auto mark = [&](int m) {
        if (ev && ev[m]) (void)hipEventRecord(ev[m], s);
    };
    if (a.pt.p < 2) return hipSuccess;
    const size_t kk = (size_t)a.pt.k * a.pt.k;
    const size_t lds = (4 * kk + 3 * (size_t)a.pt.k) * sizeof(T);
    if (tips_in_lds(a.pt.k, sizeof(T) == 4)) {
        // below K = 64 the chunk transfer matrices run beside this kernel on
        // a second stream: fewer threads here leave them CUs
        const bool wide = a.pt.k >= 64;
        auto kern = wide ? k_tips_lds<T, 1024> : k_tips_lds<T, 512>;
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        mark(0);
        hipLaunchKernelGGL(kern, dim3(a.pt.p - 1), dim3(wide ? 1024 : 512), lds, s, a);
        mark(3);
    } else {
        const int ncg = (a.pt.k + 63) / 64;
        const size_t cols = (size_t)a.pt.k * 66 * sizeof(T);    // columns + 2 factor rows: <= 134640 B
        if (cols > kMaxLds) return hipErrorInvalidValue;
        for (const void *f : {(const void *)k_tips_global_vw<T>, (const void *)k_tips_global_rinv<T>}) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols);
            if (e != hipSuccess) return e;
        }
        mark(0);
        hipLaunchKernelGGL(k_tips_global_stage<T>, dim3(a.pt.p - 1, 2), dim3(256), 0, s, a);
        mark(1);
        hipLaunchKernelGGL(k_tips_global_vw<T>, dim3(a.pt.p - 1, 2 * ncg), dim3(64), cols, s, a);
        mark(2);
        const int nt = (a.pt.k + 63) / 64;
        hipLaunchKernelGGL(k_tips_global_rbar<T>, dim3(a.pt.p - 1, nt * nt), dim3(256), 0, s, a);
        const size_t rb = kk * sizeof(T);
        if (rb + 64 <= kMaxLds) {               // + pr_sh, zero_sh
            hipError_t e = hipFuncSetAttribute((const void *)k_tips_global_lu<T, true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)rb);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_tips_global_lu<T, true>), dim3(a.pt.p - 1), dim3(kTipsLuNT), rb, s, a);
        } else {
            hipLaunchKernelGGL((k_tips_global_lu<T, false>), dim3(a.pt.p - 1), dim3(kTipsLuNT), 0, s, a);
        }
        hipLaunchKernelGGL(k_tips_global_rinv<T>, dim3(a.pt.p - 1, ncg), dim3(64), cols, s, a);
        mark(3);
    }
    return hipGetLastError();
}


template hipError_t launch_tips<float>(const TipsArgs<float> &, hipStream_t, hipEvent_t *);
template hipError_t launch_tips<double>(const TipsArgs<double> &, hipStream_t, hipEvent_t *);

}  // namespace sap
