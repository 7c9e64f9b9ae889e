// Blocked banded LU / UL of the diagonal blocks with matrix-core (MFMA)
// updates, for half-bandwidths K >= 64.
//
// The method is the one of k_factor.hip (arXiv:1509.07919, Sec. 2.2 pivot
// boosting, Sec. 3.1 LU/UL factorizations): no pivoting, a pivot p with
// |p| < tau is replaced by +-tau, the UL factorization is the LU of J A_i J
// of which only the last K x K corner is kept.  Only the order of the
// floating-point operations differs: pivots are taken 16 at a time.
//
// MI355X design.  One workgroup of 4 waves (one per SIMD, so each wave may
// hold up to 512 registers) factors one block.  After the
// pivots before j0 have been applied, the only entries still to be touched
// are those of the window of rows and columns [j0, j0 + 16*NTL) with
// NTL = ceil(K/16) + 1 (entries with |r - c| > K are exact zeros and stay
// zero).  The window is held in the matrix-core accumulator layout of 16 x 16
// tiles, NTL x NTL tiles spread over the waves' registers, in circular slots:
// tile (I, J) of the block lives in slot (I mod NTL, J mod NTL) for its whole
// lifetime, so nothing moves when the window slides by one tile per panel.
// Per panel of 16 pivots (tile index p, slot ap = p mod NTL):
//   (a) the owners copy the panel tile column and tile row into LDS;
//   (b) wave 0 factors the 16 x 16 diagonal tile (boosting each pivot);
//   (c) L21 solves X U11 = A21 (a thread per row) and U12 solves
//       L11 Y = A12 (a thread per column) by substitution;
//   (d) every trailing tile is updated in registers, A22 -= L21 U12 (4 MFMAs
//       per tile), and the panel's L columns and U rows are written out;
//   (e) the slots of the retired tile row and column receive the tiles that
//       enter the window.  They are untouched entries of A, copied from HBM
//       straight into LDS (global_load_lds, no registers) at the start of the
//       panel as 2K+1 diagonal runs of 16 consecutive band entries, then laid
//       out as tiles by all threads.
#include "sap_internal.h"
#include "dev_common.h"

namespace sap {

template <typename T> struct Acc4;
template <> struct Acc4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Acc4<double> { typedef double type __attribute__((ext_vector_type(4))); };

// D += A B for a 16 x 16 x 4 slice.  Operand layouts (lane l): A[l & 15][l >> 4]
// and B[l >> 4][l & 15].  Result: element r of lane l is D[drow][dcol] below.
__device__ __forceinline__ Acc4<float>::type mfma16(float a, float b, Acc4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Acc4<double>::type mfma16(double a, double b, Acc4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> struct DLayout;
template <> struct DLayout<float> {     // rows 4(l >> 4) .. +3 of column l & 15
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ __forceinline__ int col(int lane, int) { return lane & 15; }
};
template <> struct DLayout<double> {    // rows l >> 4, +4, +8, +12 of column l & 15
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    static __device__ __forceinline__ int col(int lane, int) { return lane & 15; }
};

constexpr int kMfmaWaves = 4;

// LDS layout: stage [2K+3][16] doubles (row 0 zero, row q+1 = diagonal q,
// row 2K+2 receives the unused half of the last copy), then in elements of T:
// PC [WR][17] panel tile column, PR [16][WR+1] panel tile row, UI [16]
// reciprocal pivots (with room to spare)
__host__ __device__ inline size_t lu_mfma_lds_bytes(int k, int ntl, size_t tsize)
{
    const int wr = 16 * ntl;
    return (size_t)(2 * k + 3) * 16 * sizeof(double) +
           ((size_t)wr * 17 + 16 * (size_t)(wr + 1) + 2 * 16 * 17) * tsize;
}

template <typename T, int NTL>
__global__ __launch_bounds__(kMfmaWaves * 64) void k_lu_mfma(LuArgs<T> a)
{
    using v4 = typename Acc4<T>::type;
    using DL = DLayout<T>;
    constexpr int NW = kMfmaWaves;
    constexpr int NT = NW * 64;
    constexpr int RPW = (NTL + NW - 1) / NW;   // slot rows per wave
    constexpr int WR = 16 * NTL;
    constexpr int PRP = WR + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double tau_sh;

    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int P = a.pt.p;
    const int ul = (int)blockIdx.x >= P;
    const int blk = ul ? (int)blockIdx.x - P : (int)blockIdx.x;
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lq = lane >> 4;
    const int CS = k + 1;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int W2 = 2 * k + 1;

    double *stage = reinterpret_cast<double *>(smem_raw);
    T *PC = reinterpret_cast<T *>(stage + (2 * k + 3) * 16);
    T *PR = PC + WR * 17;
    T *UI = PR + 16 * PRP;                       // reciprocal pivots of the panel

    if (tid == 0) {
        double m = 0.0;
        for (int c = 0; c < a.nchunk; ++c) m = fmax(m, a.partial[(int64_t)blk * a.nchunk + c]);
        tau_sh = a.boost_eps >= 0.0 ? a.boost_eps * (double)(T)m : -1.0;
    }
    if (!ul) {
        // column-form entries that would reach above the block are zero
        for (int idx = tid; idx < k * CS; idx += NT) {
            const int c = idx / CS, m = idx % CS;
            if (c < nb && m > c) {
                a.Uc[(s0 + c) * CP + m] = T(0);
                if (a.Lr) a.Lr[(s0 + c) * CP + m] = T(0);
            }
        }
    }

    // Wave w owns the slot rows sa = w + NW*ai (ai < RPW) and all NTL slot
    // columns; rows sa >= NTL (only when NW does not divide NTL) are spare
    // registers that are updated like the others and never read.
    v4 acc[RPW][NTL];
#pragma unroll
    for (int ai = 0; ai < RPW; ++ai)
#pragma unroll
        for (int b = 0; b < NTL; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[ai][b][r] = (T)block_entry(a.band, n, k, s0, nb, ul,
                                               16 * (wave + NW * ai) + DL::row(lane, r),
                                               16 * b + DL::col(lane, r));
    // offset of slot index x from the panel slot ap, i.e. tile index minus p
    auto off = [](int x, int ap) { return x >= ap ? x - ap : x - ap + NTL; };

    // entering entries of panel p: index m in [16(NTL+p), 16(NTL+p)+16);
    // stage row q+1, column s: delta = q - K, entry (m, m-delta) for delta >= 0
    // and (m+delta, m) for delta < 0, m = 16(NTL+p) + s.  One copy instruction
    // moves diagonals q = 2g, 2g+1 (lane l: q = 2g + (l >> 5), s = (l >> 1) & 15,
    // dword l & 1 of the double).  Entries past the block end are masked when
    // read; their addresses are clamped into the band array.
    const int64_t bandlen = (int64_t)W2 * n;
    auto prefetch = [&](int64_t p) {
        const int q0 = lane >> 5, ss = (lane >> 1) & 15, half = lane & 1;
        const int64_t m = 16 * (NTL + p) + ss;
        for (int g = wave; 2 * g < W2; g += NW) {
            const int q = 2 * g + q0;
            const int delta = q - k;
            const int64_t col = ul ? (s0 + nb - 1 - m + (delta > 0 ? delta : 0))
                                   : (s0 + m - (delta > 0 ? delta : 0));
            int64_t o = (int64_t)(ul ? (k - delta) : (k + delta)) * n + col;
            o = o < 0 ? 0 : (o >= bandlen ? bandlen - 1 : o);
            const unsigned *src = reinterpret_cast<const unsigned *>(a.band + o) + half;
            __builtin_amdgcn_global_load_lds(
                (const void *)src,
                (__attribute__((address_space(3))) void *)(stage + (2 * g + 1) * 16), 4, 0, 0);
        }
    };
    for (int idx = tid; idx < 16; idx += NT) stage[idx] = 0.0;

    prefetch(0);
    __syncthreads();
    const double tau_d = tau_sh;
    const T tau = (T)tau_d;
    const bool do_boost = tau_d >= 0.0;
    int nboost = 0;

    const int64_t npanel = (nb + 15) / 16;
    for (int64_t p = 0; p < npanel; ++p) {
        const int64_t j0 = 16 * p;
        const int ap = (int)(p % NTL);
        const int nact = (int)min((int64_t)16, nb - j0);

        // (a) panel tile column and tile row to LDS
#pragma unroll
        for (int ai = 0; ai < RPW; ++ai) {
            const int sa = wave + NW * ai;
            if (sa < NTL) {
                const int ro = off(sa, ap);
#pragma unroll
                for (int b = 0; b < NTL; ++b) {
                    const int co = off(b, ap);
                    if (co == 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            PC[(16 * ro + DL::row(lane, r)) * 17 + DL::col(lane, r)] = acc[ai][b][r];
                    } else if (ro == 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            PR[DL::row(lane, r) * PRP + 16 * co + DL::col(lane, r)] = acc[ai][b][r];
                    }
                }
            }
        }
        __syncthreads();

        // (b) diagonal tile: LU with boosting, lane t < 16 holding row t;
        // the reciprocal pivots go to UI[0][t] (0 for pivots past the block
        // end, which only the last panel has: their rows and columns are zero)
        if (wave == 0) {
            T row[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) row[c] = lane < 16 ? PC[lane * 17 + c] : T(0);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                if (t < nact) {
                    const T praw = lane_bcast(row[t], t);
                    T piv = praw;
                    bool boosted = false;
                    if (do_boost && fabs((double)praw) < (double)tau) {
                        piv = praw >= T(0) ? tau : -tau;
                        boosted = true;
                    }
                    if (lane == 0) {
                        nboost += boosted ? 1 : 0;
                        if (piv == T(0)) a.status[1] = 1;
                    }
                    const T rp = T(1) / piv;
                    const T l = row[t] * rp;
                    const bool below = lane > t;
#pragma unroll
                    for (int c = t + 1; c < 16; ++c)
                        row[c] = below ? fma(-l, lane_bcast(row[c], t), row[c]) : row[c];
                    row[t] = below ? l : (lane == t ? piv : row[t]);
                    if (lane == t) UI[t] = rp;
                } else if (lane == t) {
                    UI[t] = T(0);
                }
            }
            if (lane < 16)
#pragma unroll
                for (int c = 0; c < 16; ++c) PC[lane * 17 + c] = row[c];
        }
        __syncthreads();

        // (c) L21 rows solve x U11 = a (one thread per row), U12 columns solve
        // L11 y = a (one thread per column)
        for (int task = tid; task < 2 * (WR - 16); task += NT) {
            T x[16];
            if (task < WR - 16) {
                T *pr = PC + (16 + task) * 17;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    T v = pr[t];
#pragma unroll
                    for (int q = 0; q < t; ++q) v = fma(-x[q], PC[q * 17 + t], v);
                    x[t] = v * UI[t];
                }
#pragma unroll
                for (int t = 0; t < 16; ++t) pr[t] = x[t];
            } else {
                const int c = 16 + task - (WR - 16);
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    T v = PR[t * PRP + c];
#pragma unroll
                    for (int q = 0; q < t; ++q) v = fma(-PC[t * 17 + q], x[q], v);
                    x[t] = v;
                }
#pragma unroll
                for (int t = 0; t < 16; ++t) PR[t * PRP + c] = x[t];
            }
        }
        __syncthreads();

        // (d) trailing update A22 -= L21 U12 on every slot (the retired row
        // and column are overwritten in (e), so they need no exception): per
        // 4-wide slice, the wave's L21 operands (one per slot row) and U12
        // operands (one per slot column) are read once and feed RPW x NTL
        // independent MFMAs
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            T av[RPW], bv[NTL];
#pragma unroll
            for (int ai = 0; ai < RPW; ++ai) {
                const int sa = min(wave + NW * ai, NTL - 1);
                av[ai] = -PC[(16 * off(sa, ap) + lr) * 17 + 4 * s + lq];
            }
#pragma unroll
            for (int b = 0; b < NTL; ++b) bv[b] = PR[(4 * s + lq) * PRP + 16 * off(b, ap) + lr];
#pragma unroll
            for (int ai = 0; ai < RPW; ++ai)
#pragma unroll
                for (int b = 0; b < NTL; ++b) acc[ai][b] = mfma16(av[ai], bv[b], acc[ai][b]);
        }
        // outputs of pivot j = j0 + t: column-form coefficient rows
        //   Lc[j] = [1, l(j+m, j)],  Uc[j+m][m] = u(j, j+m),  Uc[j][0] = 1/u_jj
        // (and the row forms Ur, Lr), or the UL corner
        for (int t = wave; t < nact; t += NW) {
            const int64_t j = j0 + t;
            const T piv = PC[t * 17 + t];
            for (int m = lane; m < CS; m += 64) {
                const T lv = m == 0 ? T(1) : PC[(t + m) * 17 + t];
                const T uo = (t + m < 16) ? PC[t * 17 + t + m] : PR[t * PRP + t + m];
                const T uv = m == 0 ? T(1) / piv : uo;
                const bool in = j + m < nb;
                if (!ul) {
                    a.Lc[(s0 + j) * CP + m] = lv;
                    if (in) a.Uc[(s0 + j + m) * CP + m] = uv;
                    if (a.Ur) a.Ur[(s0 + j) * CP + m] = in ? uv : T(0);
                    if (a.Lr && in) a.Lr[(s0 + j + m) * CP + m] = lv;
                } else if (a.corner && j >= nb - k && in) {
                    const int64_t b0 = j - (nb - k);
                    T *cn = a.corner + (int64_t)blk * k * k;
                    if (m >= 1) cn[(b0 + m) * k + b0] = lv;
                    cn[b0 * k + b0 + m] = m == 0 ? piv : uv;
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);          // this wave's stage copies have landed
        __syncthreads();
        // (e) the tiles entering the window: tile row p + NTL (columns
        // p+1 .. p+NTL) into PR, tile column p + NTL (rows p+1 .. p+NTL-1) into
        // PC.  Entry (gr, gc) (relative to j0) is stage row gr - gc + K + 1
        // (row 0, zero, when |gr - gc| > K), column max(gr, gc) - 16 NTL; zero
        // past the block end.
        for (int e = tid; e < 16 * WR + 16 * (WR - 16); e += NT) {
            int gr, gc;
            T *dst;
            if (e < 16 * WR) {
                const int rr = e / WR, cc = e - rr * WR;
                gr = 16 * NTL + rr;
                gc = 16 + cc;
                dst = PR + rr * PRP + cc;
            } else {
                const int f = e - 16 * WR;
                const int rr = f >> 4, cc = f & 15;
                gr = 16 + rr;
                gc = 16 * NTL + cc;
                dst = PC + rr * 17 + cc;
            }
            const int dl = gr - gc;
            const int mx = max(gr, gc);
            const int srow = (dl >= -k && dl <= k) ? dl + k + 1 : 0;
            const double v = stage[srow * 16 + mx - 16 * NTL];
            *dst = (j0 + mx < nb) ? (T)v : T(0);
        }
        __syncthreads();
        // the owners put them into the slots of the retired tile row and
        // column as the product I E (4 MFMAs from a zero accumulator), so the
        // accumulators are only ever produced by MFMAs and stay in AGPRs
        {
            const v4 zero = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int ai = 0; ai < RPW; ++ai) {
                const int sa = wave + NW * ai;
                if (sa < NTL) {
                    const int ro = off(sa, ap);
#pragma unroll
                    for (int b = 0; b < NTL; ++b) {
                        const int co = off(b, ap);
                        if (ro == 0 || co == 0) {
                            v4 d = zero;
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                // B operand E[4s + lq][lr]; A operand identity
                                const T e = ro == 0 ? PR[(4 * s + lq) * PRP + 16 * (co == 0 ? NTL - 1 : co - 1) + lr]
                                                    : PC[(16 * (ro - 1) + 4 * s + lq) * 17 + lr];
                                const T id = (lr == 4 * s + lq) ? T(1) : T(0);
                                d = mfma16(id, e, d);
                            }
                            acc[ai][b] = d;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (p + 1 < npanel) prefetch(p + 1);
    }
    if (tid == 0 && nboost) atomicAdd(&a.status[0], nboost);
}

template <typename T, int NTL>
static hipError_t launch_lu_mfma_ntl(const LuArgs<T> &a, hipStream_t s)
{
    const size_t lds = lu_mfma_lds_bytes(a.pt.k, NTL, sizeof(T));
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_lu_mfma<T, NTL>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid(a.with_ul ? 2 * a.pt.p : a.pt.p);
    hipLaunchKernelGGL(kern, grid, dim3(kMfmaWaves * 64), lds, s, a);
    return hipGetLastError();
}

// The window needs 16 (NTL - 1) >= K; a larger NTL only adds zero tiles, so
// a few window sizes cover every K.  Up to K = 208 (14 x 14 tiles) the window
// fits the 512 registers per lane of a wave alone on its SIMD for FP32
// factors.  FP64 windows take twice the registers: above K = 96 part of the
// window spills to scratch, and the 14 x 14 window (K > 160) leaves too few
// registers for the rest of the kernel, so FP64 stops at 11 x 11 tiles.
bool lu_mfma_supported(int k, bool fp32) { return k >= 1 && k <= (fp32 ? 208 : 160); }

template <typename T>
hipError_t launch_lu_mfma(const LuArgs<T> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (!lu_mfma_supported(k, sizeof(T) == 4)) return hipErrorInvalidValue;
    const int ntl = (k + 15) / 16 + 1;
    if (ntl <= 2) return launch_lu_mfma_ntl<T, 2>(a, s);
    if (ntl <= 3) return launch_lu_mfma_ntl<T, 3>(a, s);
    if (ntl <= 4) return launch_lu_mfma_ntl<T, 4>(a, s);
    if (ntl <= 5) return launch_lu_mfma_ntl<T, 5>(a, s);
    if (ntl <= 7) return launch_lu_mfma_ntl<T, 7>(a, s);
    if (ntl <= 9) return launch_lu_mfma_ntl<T, 9>(a, s);
    if (ntl <= 11) return launch_lu_mfma_ntl<T, 11>(a, s);
    if constexpr (sizeof(T) == 4) return launch_lu_mfma_ntl<T, 14>(a, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_lu_mfma<float>(const LuArgs<float> &, hipStream_t);
template hipError_t launch_lu_mfma<double>(const LuArgs<double> &, hipStream_t);

}  // namespace sap
