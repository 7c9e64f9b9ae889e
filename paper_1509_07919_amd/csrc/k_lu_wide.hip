// Banded LU / UL of the diagonal blocks for FP64 factors of very wide bands
// (K > 160), whose (K+B)^2 active window fits neither one CU's registers
// beside the rest of a kernel nor its LDS.
//
// The method is the one of k_factor.hip (arXiv:1509.07919, Sec. 2.2 pivot
// boosting, Sec. 3.1 LU/UL factorizations): no pivoting, a pivot p with
// |p| < tau is replaced by +-tau, the UL factorization is the LU of J A_i J
// of which only the last K x K corner is kept.  Pivots are taken B at a time.
//
// MI355X design.  One workgroup of 256 threads factors one block (LU and UL
// of all blocks in one launch).  The window -- rows and columns j0 ..
// j0+WM-1 of the block, WM = K + B -- lives in a per-workgroup slab of the
// workspace as a circular WM x WM array: entry (r, c) sits in slot
// (r mod WM, c mod WM) for its whole lifetime, so sliding the window by B
// only overwrites the slots of the retired rows and columns with entering
// entries of A.  Per panel of B pivots:
//   (a) the panel columns (WM x B) and the panel rows right of them (B x K)
//       are copied into LDS;
//   (b) all threads factor the panel right-looking in LDS, one barrier per
//       pivot (row multipliers in parallel over the WM rows, the U12 rows by
//       the same elimination, so L11^{-1} A12 needs no separate solve);
//   (c) the panel's L columns and U rows are written out;
//   (d) the trailing window A22 -= L21 U12 is updated in place, thread c
//       owning window column c: its B values of U12 stay in registers and
//       the B multipliers of each row are LDS broadcasts, so every FP64 FMA
//       costs one global read-modify-write per B FMAs (coalesced across the
//       columns of a row);
//   (e) the entering rows and columns of the next window are read from A.
// The window slab (about 660 KB per workgroup at K = 255) stays in the
// 256 MB last-level cache across panels.
#include "sap_internal.h"
#include "dev_common.h"

namespace sap {

constexpr int kWideB = 32;          // pivots per panel
constexpr int kWideNT = 256;        // threads per workgroup

__host__ __device__ inline int wide_wm(int k) { return k + kWideB; }

size_t lu_wide_window_bytes(int k) { return (size_t)wide_wm(k) * wide_wm(k) * sizeof(double); }

__global__ __launch_bounds__(kWideNT) void k_lu_wide(LuArgs<double> a, double *slabs)
{
    constexpr int B = kWideB;
    constexpr int NT = kWideNT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double tau_sh, inv_sh;

    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int P = a.pt.p;
    const int ul = (int)blockIdx.x >= P;
    const int blk = ul ? (int)blockIdx.x - P : (int)blockIdx.x;
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int CS = k + 1;
    const int CP = coef_pitch(k, (int)sizeof(double));   // row pitch in HBM
    const int WM = wide_wm(k);
    const int LP = B + 1;                                // LDS pitch of the panel columns
    double *win = slabs + (int64_t)blockIdx.x * WM * WM; // circular window
    double *Lp = reinterpret_cast<double *>(smem_raw);   // [WM][B+1] panel columns
    double *Up = Lp + (size_t)WM * LP;                   // [B][K] panel rows right of the panel
    double *UI = Up + (size_t)B * k;                     // [B] reciprocal pivots

    auto slot = [&](int64_t r, int64_t c) -> double & {
        return win[(r % WM) * WM + (c % WM)];
    };

    if (tid == 0) {
        double m = 0.0;
        for (int c = 0; c < a.nchunk; ++c) m = fmax(m, a.partial[(int64_t)blk * a.nchunk + c]);
        tau_sh = a.boost_eps >= 0.0 ? a.boost_eps * m : -1.0;
    }
    if (!ul) {
        // column-form entries that would reach above the block are zero
        for (int idx = tid; idx < k * CS; idx += NT) {
            const int c = idx / CS, m = idx % CS;
            if (c < nb && m > c) {
                a.Uc[(s0 + c) * CP + m] = 0.0;
                if (a.Lr) a.Lr[(s0 + c) * CP + m] = 0.0;
            }
        }
    }
    // the first window: rows and columns 0 .. WM-1 of the block
    for (int64_t idx = tid; idx < (int64_t)WM * WM; idx += NT) {
        const int64_t r = idx / WM, c = idx % WM;
        slot(r, c) = block_entry(a.band, n, k, s0, nb, ul, r, c);
    }
    __threadfence_block();
    __syncthreads();
    const double tau = tau_sh;
    const bool do_boost = tau >= 0.0;
    int nboost = 0;
    bool zero_piv = false;

    const int64_t npanel = (nb + B - 1) / B;
    for (int64_t pnl = 0; pnl < npanel; ++pnl) {
        const int64_t j0 = pnl * B;
        const int nact = (int)min((int64_t)B, nb - j0);
        // (a) panel columns j0 .. j0+B-1 (window rows 0..WM-1) and the rows
        // j0 .. j0+B-1 to their right (window columns B..WM-1)
        for (int idx = tid; idx < WM * B; idx += NT) {
            const int r = idx / B, c = idx % B;
            Lp[r * LP + c] = slot(j0 + r, j0 + c);
        }
        for (int idx = tid; idx < B * k; idx += NT) {
            const int r = idx / k, c = idx % k;
            Up[r * k + c] = slot(j0 + r, j0 + B + c);
        }
        __syncthreads();
        // (b) right-looking elimination of the panel's pivots in LDS
        for (int t = 0; t < nact; ++t) {
            if (tid == 0) {
                const double praw = Lp[t * LP + t];
                double piv = praw;
                if (do_boost && fabs(praw) < tau) {
                    piv = praw >= 0.0 ? tau : -tau;
                    ++nboost;
                }
                if (piv == 0.0) zero_piv = true;
                Lp[t * LP + t] = piv;
                inv_sh = 1.0 / piv;
                UI[t] = inv_sh;
            }
            __syncthreads();
            const double inv = inv_sh;
            // multipliers l_rt (rows t+1 .. WM-1) and their updates of the
            // panel columns t+1 .. B-1
            for (int r = t + 1 + tid; r < WM; r += NT) {
                const double l = Lp[r * LP + t] * inv;
                Lp[r * LP + t] = l;
                for (int c = t + 1; c < B; ++c) Lp[r * LP + c] = fma(-l, Lp[t * LP + c], Lp[r * LP + c]);
            }
            __syncthreads();
            // the same elimination on the rows right of the panel: row r of
            // U12 (r = t+1 .. B-1) loses l_rt times row t
            for (int idx = tid; idx < (B - 1 - t) * k; idx += NT) {
                const int r = t + 1 + idx / k, c = idx % k;
                Up[r * k + c] = fma(-Lp[r * LP + t], Up[t * k + c], Up[r * k + c]);
            }
            __syncthreads();
        }
        // (c) outputs of pivot j = j0 + t: the column-form rows Lc[j],
        // Uc[j+m][m] = u(j, j+m), Uc[j][0] = 1/u_jj (and Ur, Lr), or the
        // UL corner
        for (int idx = tid; idx < nact * CS; idx += NT) {
            const int t = idx / CS, m = idx % CS;
            const int64_t j = j0 + t;
            const double piv = Lp[t * LP + t];
            const double lv = m == 0 ? 1.0 : Lp[(t + m) * LP + t];
            const double uo = (t + m < B) ? Lp[t * LP + t + m] : Up[t * k + (t + m - B)];
            const double uv = m == 0 ? UI[t] : uo;
            const bool in = j + m < nb;
            if (!ul) {
                a.Lc[(s0 + j) * CP + m] = in || m == 0 ? lv : 0.0;
                if (in) a.Uc[(s0 + j + m) * CP + m] = uv;
                if (a.Ur) a.Ur[(s0 + j) * CP + m] = in ? uv : 0.0;
                if (a.Lr && in) a.Lr[(s0 + j + m) * CP + m] = lv;
            } else if (a.corner && j >= nb - k && in) {
                const int64_t b0 = j - (nb - k);
                double *cn = a.corner + (int64_t)blk * k * k;
                if (m >= 1) cn[(b0 + m) * k + b0] = lv;
                cn[b0 * k + b0 + m] = m == 0 ? piv : uv;
            }
        }
        // (d) trailing update of window rows and columns B .. WM-1 (thread
        // c owns column B + c), then (e) the entering entries
        if (pnl + 1 < npanel) {
            for (int c = tid; c < k; c += NT) {
                double u[B];
#pragma unroll
                for (int t = 0; t < B; ++t) u[t] = t < nact ? Up[t * k + c] : 0.0;
                const int64_t gc = j0 + B + c;
                // rows in groups of RG: their window reads are in flight together
                constexpr int RG = 8;
                int r = 0;
                for (; r + RG <= k; r += RG) {
                    double v[RG];
#pragma unroll
                    for (int q = 0; q < RG; ++q) v[q] = slot(j0 + B + r + q, gc);
#pragma unroll
                    for (int q = 0; q < RG; ++q) {
                        const double *lr = Lp + (B + r + q) * LP;
                        double v2 = 0.0;
#pragma unroll
                        for (int t = 0; t < B; t += 2) {
                            v[q] = fma(-lr[t], u[t], v[q]);
                            v2 = fma(-lr[t + 1], u[t + 1], v2);
                        }
                        v[q] += v2;
                    }
#pragma unroll
                    for (int q = 0; q < RG; ++q) slot(j0 + B + r + q, gc) = v[q];
                }
                for (; r < k; ++r) {
                    const double *lr = Lp + (B + r) * LP;
                    double v = slot(j0 + B + r, gc);
                    double v2 = 0.0;
#pragma unroll
                    for (int t = 0; t < B; t += 2) {
                        v = fma(-lr[t], u[t], v);
                        v2 = fma(-lr[t + 1], u[t + 1], v2);
                    }
                    slot(j0 + B + r, gc) = v + v2;
                }
            }
            // entering rows j0+WM .. j0+WM+B-1 (columns j0+B .. j0+WM+B-1)
            // and entering columns (rows j0+B .. j0+WM-1): untouched entries
            // of A, into the slots of the retired rows and columns
            const int64_t e0 = j0 + WM;
            for (int idx = tid; idx < B * WM; idx += NT) {
                const int64_t r = e0 + idx / WM, c = j0 + B + idx % WM;
                slot(r, c) = block_entry(a.band, n, k, s0, nb, ul, r, c);
            }
            for (int idx = tid; idx < k * B; idx += NT) {
                const int64_t r = j0 + B + idx / B, c = e0 + idx % B;
                slot(r, c) = block_entry(a.band, n, k, s0, nb, ul, r, c);
            }
        }
        __threadfence_block();                 // the window writes, to the next panel's reads
        __syncthreads();
    }
    if (tid == 0 && nboost) atomicAdd(&a.status[0], nboost);
    if (tid == 0 && zero_piv) a.status[1] = 1;
}

size_t lu_wide_lds_bytes(int k)
{
    return ((size_t)wide_wm(k) * (kWideB + 1) + (size_t)kWideB * k + kWideB) * sizeof(double);
}

hipError_t launch_lu_wide(const LuArgs<double> &a, double *slabs, hipStream_t s)
{
    const size_t lds = lu_wide_lds_bytes(a.pt.k);
    if (lds > kMaxLds || !slabs) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)k_lu_wide,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid(a.with_ul ? 2 * a.pt.p : a.pt.p);
    hipLaunchKernelGGL(k_lu_wide, grid, dim3(kWideNT), lds, s, a, slabs);
    return hipGetLastError();
}

}  // namespace sap
