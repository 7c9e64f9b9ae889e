// Block norms and the banded LU / UL factorization of the diagonal blocks.
//
// LU without pivoting but with pivot boosting (arXiv:1509.07919, Sec. 2.2
// pivot-boosting paragraph; Sec. 3.1 "LU/UL factorizations"): for each block
// A_i, for j = 0..N_i-1: p = a_jj, boosted to +-tau when |p| < tau; the
// multipliers l_rj = a_rj / p and the update a_rc -= l_rj a_jc touch only the
// (K+1) x (K+1) window of rows and columns j..j+K.  The UL factorization of
// A_i is the LU of J A_i J (J reverses row/column order); only the last K
// steps of it -- the top-left corner of the UL factors -- are written.
//
// MI355X design.  One workgroup factors one block (P workgroups for LU, P
// more for UL run concurrently).  The active window lives in VGPRs as a
// circular WC x WC ring (WC >= K+1, a power of two): entry (r, c) of the
// block sits in ring slot (r mod WC, c mod WC) for its whole lifetime, so
// nothing moves when the window slides.  Lanes own ring columns, waves own
// strided sets of ring rows; each thread rotates its register array after
// publishing a pivot row, so all register indices are static and the step
// loop needs no unrolling.  Per step: the owners of the pivot row and
// column publish them to LDS (double-buffered by step parity), one barrier,
// then every thread applies the rank-1 update to all its slots.  Entries
// outside the band are exact zeros, so the update needs no masking and never
// creates fill.  The row and column that enter the ring after step j are
// untouched originals; they are streamed from HBM in chunks of S indices
// (2K+1 diagonal segments, each a coalesced run) into double-buffered LDS,
// one chunk ahead of use.
#include "sap_internal.h"
#include "dev_common.h"

namespace sap {


// ---------------------------------------------------------------- norms

// partial[blk][chunk] = max |a_rc| over the columns of one 64-column chunk
// of diagonal block blk (rows restricted to the block).  Lane l of wave w
// takes column l of the chunk and the diagonals q = w (mod 4): each wave
// load is one coalesced 512-byte run of a diagonal, and 4 times as many
// workgroups as columns / 256 keep enough loads in flight for HBM.
__global__ __launch_bounds__(256) void k_block_norm(const double *__restrict__ band,
                                                    Partition pt,
                                                    double *__restrict__ partial,
                                                    int nchunk, int *__restrict__ status)
{
    // the factorization's status words start at zero (the LU and tips
    // kernels that follow count boosted pivots and flag singularity)
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < kStatusWords) status[threadIdx.x] = 0;
    const int blk = blockIdx.y;
    const int64_t s0 = pt.starts[blk];
    const int64_t nb = pt.starts[blk + 1] - s0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t x = (int64_t)blockIdx.x * 64 + lane;
    double m = 0.0;
    if (x < nb) {
        const int64_t c = s0 + x;
        for (int q = wave; q <= 2 * pt.k; q += 4) {
            const int64_t r = x + q - pt.k;
            if (r >= 0 && r < nb) m = fmax(m, fabs(band[(int64_t)q * pt.n + c]));
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blk * nchunk + blockIdx.x] = red[0];
}

hipError_t launch_block_norm(const double *band, const Partition &pt, double *partial,
                             int nchunk, int *status, hipStream_t s)
{
    dim3 grid(nchunk, pt.p);
    hipLaunchKernelGGL(k_block_norm, grid, dim3(256), 0, s, band, pt, partial, nchunk, status);
    return hipGetLastError();
}

// ------------------------------------------------------------------- LU

// Entry (r, c) of the block as seen by the LU (ul = 0) or by the LU of the
// reversed block (ul = 1); 0 outside the block or the band.

template <typename T, int WC, int S, int NT>
__global__ __launch_bounds__(NT) void k_banded_lu(LuArgs<T> a)
{
    constexpr int RS = NT / WC;          // ring-row sets
    constexpr int RPT = WC / RS;         // ring rows per thread
    static_assert(NT % WC == 0 && WC % RS == 0, "bad ring shape");
    constexpr int KMAX = WC - 1;
    constexpr int PR = ((2 * KMAX + 1) * S + NT - 1) / NT;   // prefetch regs

    // stage buffer b: rows q = -1..2K+1 of S entries at stage + b*stage_sz +
    // (q+1)*S; rows -1 and 2K+1 stay zero, so clamped row indices need no mask
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *stage = reinterpret_cast<T *>(smem_raw);               // [2][(2K+3)*S]
    T *obuf = stage + 2 * (2 * a.pt.k + 3) * S;               // [S][2][K+1]
    __shared__ __align__(16) T lcol[2][WC];                   // perm: [rs*RPT+i]
    __shared__ __align__(16) T urow[2][WC];
    __shared__ double tau_sh;

    const int k = a.pt.k;
    const int64_t n = a.pt.n;
    const int P = a.pt.p;
    const int ul = (int)blockIdx.x >= P;
    const int blk = ul ? (int)blockIdx.x - P : (int)blockIdx.x;
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int sc = tid % WC;
    const int rs = tid / WC;
    const int CS = k + 1;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int W2 = 2 * k + 1;
    const int stage_sz = (W2 + 2) * S;

    // boost threshold tau = eps * max|A_i| (in the factor precision)
    if (tid == 0) {
        double m = 0.0;
        for (int c = 0; c < a.nchunk; ++c) m = fmax(m, a.partial[(int64_t)blk * a.nchunk + c]);
        tau_sh = a.boost_eps >= 0.0 ? a.boost_eps * (double)(T)m : -1.0;
    }

    // LU direction: zero the coefficient slots that would point above row 0
    if (!ul) {
        for (int idx = tid; idx < k * CS; idx += NT) {
            const int c = idx / CS, m = idx % CS;       // column c < K, slot m
            if (c < nb && m > c) {
                a.Uc[(s0 + c) * CP + m] = T(0);
                if (a.Lr) a.Lr[(s0 + c) * CP + m] = T(0);
            }
        }
    }

    // initial ring: rows/cols 0..WC-1
    T w[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
        w[i] = (T)block_entry(a.band, n, k, s0, nb, ul, rs + RS * i, sc);

    // chunk prefetch: entering index m = WC + t*S + s; slot f = q*S + s with
    // q = delta + K; delta >= 0 -> entry (m, m-delta), delta < 0 -> (m+delta, m).
    // For a fixed q the S entries are consecutive band elements (ascending
    // for the LU, descending for the UL): a coalesced run.
    double pre[PR];                 // raw band values (converted at commit)
    auto prefetch = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            const int q = f / S, ss = f % S;              // S is a power of two
            const int delta = q - k;
            const int64_t m = WC + t * S + ss;
            double v = 0.0;
            if (f < W2 * S && m < nb) {  // m > K >= |delta|: other index >= 0
                const int64_t base = (int64_t)(ul ? (k - delta) : (k + delta)) * n;
                const int64_t col = ul ? (s0 + nb - 1 - m + (delta > 0 ? delta : 0))
                                       : (s0 + m - (delta > 0 ? delta : 0));
                v = a.band[base + col];
            }
            pre[i] = v;
        }
    };
    auto commit = [&](int64_t t) {
        T *dst = stage + (t & 1) * stage_sz + S;
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            if (f < W2 * S) dst[f] = (T)pre[i];
        }
    };
    for (int idx = tid; idx < 4 * S; idx += NT) {          // the zero rows
        const int bsel = idx / (2 * S), r = (idx / S) & 1, c = idx % S;
        stage[bsel * stage_sz + (r ? (W2 + 1) * S : 0) + c] = T(0);
    }
    // Outputs of one chunk of S steps (L column and U row of each step) are
    // kept in LDS and written out by all threads at the next chunk boundary,
    // so no global access is pending between boundaries.
    auto flush = [&](int64_t j0) {
        if (ul) return;
        const int tot = S * CS;
        for (int idx = tid; idx < tot; idx += NT) {
            const int jj = idx / CS, m = idx - jj * CS;
            const int64_t j = j0 + jj;
            if (j >= nb) continue;
            const T lv = obuf[jj * 2 * CS + m];
            const T uv = obuf[jj * 2 * CS + CS + m];
            const bool in = j + m < nb;
            a.Lc[(s0 + j) * CP + m] = lv;
            if (in) a.Uc[(s0 + j + m) * CP + m] = uv;
            if (a.Ur) a.Ur[(s0 + j) * CP + m] = in ? uv : T(0);
            if (a.Lr && in) a.Lr[(s0 + j + m) * CP + m] = lv;
        }
    };
    prefetch(0);
    __syncthreads();
    // Drain the ring-fill loads here: otherwise the wait for them is placed
    // inside the step loop, where it also waits for every pending store.
    __builtin_amdgcn_s_waitcnt(0);
    const double tau_d = tau_sh;
    const T tau = (T)tau_d;
    const bool do_boost = tau_d >= 0.0;
    int nboost = 0;

    // Thread (rs, sc) owns ring rows rs + RS*i.  It publishes them as pivot
    // rows in the order i = 0, 1, ..., so after each publish it rotates w[]
    // left by one: its next pivot row is always w[0], and register i holds
    // ring row rs + RS*((i + rot) mod RPT).
    int rot = 0;
    for (int64_t j = 0; j < nb; ++j) {
        const int u = (int)(j & (WC - 1));
        const bool own_row = rs == (u % RS);         // holds ring row u in w[0]
        T *ur = urow[u & 1];
        T *lc = lcol[u & 1];
        const int lbase = rs * RPT;
        if ((j & (S - 1)) == 0) {                     // chunk boundary
            commit(j / S);                            // entering data of this chunk
            if (j > 0) flush(j - S);                  // outputs of the last chunk
        }
        // phase A: publish pivot row (by ring column) and pivot column
        if (own_row) ur[sc] = w[0];
        if (sc == u) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) lc[lbase + ((i + rot) & (RPT - 1))] = w[i];
        }
        __syncthreads();
        // phase B
        const T praw = ur[u];
        T piv = praw;
        bool boosted = false;
        if (do_boost && fabs((double)praw) < (double)tau) {
            piv = praw >= T(0) ? tau : -tau;
            boosted = true;
        }
        if (tid == 0) {
            nboost += boosted ? 1 : 0;
            if (piv == T(0)) a.status[1] = 1;
        }
        const T inv = T(1) / piv;
        const T ucs = ur[sc] * inv;
#pragma unroll
        for (int i = 0; i < RPT; ++i) w[i] = fma(-lc[lbase + ((i + rot) & (RPT - 1))], ucs, w[i]);

        // outputs: thread t = m handles offset m of row/column j
        if (tid <= k) {
            const int m = tid;
            const int sl = (u + m) & (WC - 1);               // ring slot of j+m
            const T lv = m == 0 ? T(1) : lc[(sl % RS) * RPT + sl / RS] * inv;
            const T uv = m == 0 ? inv : ur[sl];
            const bool in = j + m < nb;
            if (!ul) {
                T *ob = obuf + (j & (S - 1)) * 2 * CS;
                ob[m] = lv;
                ob[CS + m] = uv;
            } else if (a.corner && j >= nb - k && in) {
                const int64_t b0 = j - (nb - k);
                T *cn = a.corner + (int64_t)blk * k * k;
                if (m >= 1) cn[(b0 + m) * k + b0] = lv;
                cn[b0 * k + b0 + m] = m == 0 ? piv : uv;
            }
        }

        // entering row and column j+WC replace ring slot u
        // (row q of the stage holds delta = q - K; out-of-band deltas are
        // clamped onto the zero rows -1 and 2K+1)
        const T *stg = stage + ((j / S) & 1) * stage_sz + S;
        const int so = (int)(j & (S - 1));
        if (own_row) {
            const int dc = (sc - u - 1) & (WC - 1);          // col = j+1+dc
            const int delta = WC - 1 - dc;                   // (j+WC) - col >= 0
            w[0] = stg[min(delta + k, W2) * S + so];
        }
        if (sc == u) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int sr = rs + RS * ((i + rot) & (RPT - 1));
                const int dr = (sr - u - 1) & (WC - 1);
                const int delta = WC - 1 - dr;               // (j+WC) - row >= 0
                w[i] = stg[max(k - delta, -1) * S + so];
            }
        }
        if (own_row) {
            const T t0 = w[0];
#pragma unroll
            for (int i = 0; i < RPT - 1; ++i) w[i] = w[i + 1];
            w[RPT - 1] = t0;
            rot = (rot + 1) & (RPT - 1);
        }
        if ((j & (S - 1)) == 0) prefetch(j / S + 1);
    }
    __syncthreads();
    flush((nb - 1) & ~(int64_t)(S - 1));              // last (partial) chunk
    if (tid == 0 && nboost) atomicAdd(&a.status[0], nboost);
}

// ------------------------------------------------------------ blocked LU
//
// The same factorization, B pivots per panel.  The active window of the block
// -- rows and columns j0 .. j0+K+B-1 -- is a (K+B) x (K+B) array in LDS,
// double-buffered.  On entering panel p its first B columns are factored and
// its U12 = L11^{-1} A12 is formed.  Per panel (two barriers):
//   1. all threads form the next window's first B columns and first B rows
//      (the rank-B Schur update A22 -= L21 U12 restricted to them, entering
//      entries elsewhere);
//   2. wave 0 factors the next panel in registers (one row per lane, pivot
//      rows broadcast with v_readlane, the same boosting rule) and forms its
//      U12, while the other waves apply the rest of the update, writing
//      straight into the other buffer shifted by (B, B) so the window slides
//      for free, copy the entering rows and columns from the LDS stage, and
//      write the panel's L columns and U rows to HBM (look-ahead: the panel
//      factorization and U12 are off the critical path).
// Row r of block i appears at window row r - j0 for the LU; the UL runs the
// same code on the reversed block.
template <typename T, int B, int S, int NT, int RPL>
__global__ __launch_bounds__(NT) void k_banded_lu_blk(LuArgs<T> a)
{
    static_assert(S % B == 0, "chunks hold whole panels");
    constexpr int KMAX = 64 * RPL - B;          // window K + B fits RPL rows per lane
    constexpr int NW = NT / 64;
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
    const int lane = tid & 63, wave = tid >> 6;
    const int CS = k + 1;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int KB = k + B;                       // window size
    const int WP = KB + 1;                      // LDS pitch (odd: no bank conflicts on columns)
    const int W2 = 2 * k + 1;
    const int stage_sz = (W2 + 2) * S;

    T *win0 = reinterpret_cast<T *>(smem_raw);  // [2][KB][WP]
    T *stage = win0 + 2 * KB * WP;              // [2][(2K+3)][S], zero rows at q = -1, 2K+1
    T *uiw = stage + 2 * stage_sz;              // [2][B] 1/pivot of each window's panel

    if (tid == 0) {
        double m = 0.0;
        for (int c = 0; c < a.nchunk; ++c) m = fmax(m, a.partial[(int64_t)blk * a.nchunk + c]);
        tau_sh = a.boost_eps >= 0.0 ? a.boost_eps * (double)(T)m : -1.0;
    }
    if (!ul) {
        for (int idx = tid; idx < k * CS; idx += NT) {
            const int c = idx / CS, m = idx % CS;
            if (c < nb && m > c) {
                a.Uc[(s0 + c) * CP + m] = T(0);
                if (a.Lr) a.Lr[(s0 + c) * CP + m] = T(0);
            }
        }
    }
    // initial window: rows/cols 0 .. KB-1
    for (int idx = tid; idx < KB * KB; idx += NT) {
        const int r = idx / KB, c = idx % KB;
        win0[r * WP + c] = (T)block_entry(a.band, n, k, s0, nb, ul, r, c);
    }
    // entering index e >= 0 is global index m = KB + e; chunk t stages
    // e in [t*S, t*S+S): stage[(q+1)*S + s] = entry (m, m-delta) for delta >= 0
    // or (m+delta, m) for delta < 0, delta = q - K
    constexpr int PR = ((2 * KMAX + 1) * S + NT - 1) / NT;
    const int nitems = W2 * S;
    double pre[PR];                 // raw band values (converted at commit)
    auto prefetch = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            const int q = f / S, ss = f % S;
            const int delta = q - k;
            const int64_t m = KB + t * S + ss;
            double v = 0.0;
            if (f < nitems && m < nb) {       // m >= KB > K >= |delta|
                const int64_t base = (int64_t)(ul ? (k - delta) : (k + delta)) * n;
                const int64_t col = ul ? (s0 + nb - 1 - m + (delta > 0 ? delta : 0))
                                       : (s0 + m - (delta > 0 ? delta : 0));
                v = a.band[base + col];
            }
            pre[i] = v;
        }
    };
    auto commit = [&](int64_t t) {
        T *dst = stage + (t & 1) * stage_sz + S;
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            if (f < nitems) dst[f] = (T)pre[i];
        }
    };
    for (int idx = tid; idx < 4 * S; idx += NT) {
        const int bsel = idx / (2 * S), r = (idx / S) & 1, c = idx % S;
        stage[bsel * stage_sz + (r ? (W2 + 1) * S : 0) + c] = T(0);
    }
    prefetch(0);
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(0);
    const double tau_d = tau_sh;
    const T tau = (T)tau_d;
    const bool do_boost = tau_d >= 0.0;
    int nboost = 0;

    const int64_t npanel = (nb + B - 1) / B;
    bool zero_piv = false;
    // factorization of one panel held in wave 0's registers: row lane + 64x,
    // columns 0..B-1; the first nact_ columns are pivots.  Per pivot t the
    // pivot row is broadcast first (v_readlane; it is final once pivot t-1
    // is applied), the reciprocal comes from fast_recip, and lanes at or above
    // the pivot row take a zero multiplier instead of a branch.  ui[t]
    // receives 1/pivot.
    auto factor_panel = [&](T (&pv)[RPL][B], int nact_, T *ui) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            if (t < nact_) {
                T urow[B];
#pragma unroll
                for (int c = t; c < B; ++c) urow[c] = lane_bcast(pv[0][c], t);
                const T praw = urow[t];
                const bool boosted = do_boost && fabs((double)praw) < (double)tau;
                const T piv = boosted ? (praw >= T(0) ? tau : -tau) : praw;
                nboost += boosted ? 1 : 0;
                zero_piv = zero_piv || piv == T(0);
                const T inv = fast_recip(piv);
#pragma unroll
                for (int x = 0; x < RPL; ++x) {
                    const int rr = lane + 64 * x;
                    const T l = pv[x][t] * inv;
                    const T lm = rr > t ? l : T(0);
#pragma unroll
                    for (int c = t + 1; c < B; ++c) pv[x][c] = fma(-lm, urow[c], pv[x][c]);
                    pv[x][t] = rr > t ? l : (rr == t ? piv : pv[x][t]);
                }
                if (lane == t) ui[t] = inv;
            }
        }
    };
    // Per-thread work items that are the same for every panel.
    //   3L (all threads): the next window's first B columns (rows 0..KB-1)
    //     and first B rows (columns B..KB-1).  An entry (r, c) of the next
    //     window is a Schur update of the current window's (B+r, B+c) when
    //     r, c < K, else an entering entry of A.  Kept as (window offset,
    //     current-window row offset and column for the Schur update, or the
    //     stage offset less the panel's offset inside its chunk).
    //   3b (update waves): the other entering entries of the next window,
    //     rows max(K, B)..KB-1 x columns B..KB-1 and rows B..K-1 x columns
    //     max(K, B)..KB-1, as (window offset, stage offset).
    //   3c (update waves): (pivot t, offset m) of the outputs.
    constexpr int NIL = ((KMAX + B) * B + B * KMAX + NT - 1) / NT;
    constexpr int NTR_ = NT - 64;
    constexpr int NIB = (2 * B * KMAX + NTR_ - 1) / NTR_;
    constexpr int NIC = (B * (KMAX + 1) + NTR_ - 1) / NTR_;
    int il_dst[NIL], il_row[NIL], il_col[NIL];   // il_row < 0: entering, stage offset -1-il_row-S
    int eb_dst[NIB], eb_src[NIB], oc_t[NIC], oc_m[NIC];
    {
#pragma unroll
        for (int i = 0; i < NIL; ++i) {
            const int idx = tid + NT * i;
            il_dst[i] = -1;
            il_row[i] = il_col[i] = 0;
            if (idx < KB * B + B * k) {
                int r, c;
                if (idx < KB * B) { r = idx / B; c = idx % B; }
                else { const int q2 = idx - KB * B; r = q2 / k; c = B + q2 % k; }
                il_dst[i] = r * WP + c;
                if (r < k && c < k) {
                    il_row[i] = (B + r) * WP;
                    il_col[i] = B + c;
                } else {
                    // stage offset + S >= 0 (row q = -1 is the zero row)
                    const int qrow = min(max(r - c + k, -1), W2);
                    il_row[i] = -1 - ((qrow + 1) * S + max(r, c) - k);
                }
            }
        }
        const int tr = tid - 64;
        const int rlo = max(k, B), mkb = min(k, B);
        const int na = mkb * k, nbb = max(0, k - B) * mkb;
#pragma unroll
        for (int i = 0; i < NIB; ++i) {
            const int idx = tr + NTR_ * i;
            eb_dst[i] = -1;
            eb_src[i] = 0;
            if (tr >= 0 && idx < na + nbb) {
                int r, c;
                if (idx < na) { r = rlo + idx / k; c = B + idx % k; }
                else { const int q2 = idx - na; r = B + q2 / mkb; c = rlo + q2 % mkb; }
                const int qrow = min(max(r - c + k, -1), W2);
                eb_dst[i] = r * WP + c;
                eb_src[i] = qrow * S + max(r, c) - k;
            }
        }
#pragma unroll
        for (int i = 0; i < NIC; ++i) {
            const int idx = tr + NTR_ * i;
            const bool ok = tr >= 0 && idx < B * CS;
            oc_t[i] = ok ? idx / CS : B;      // t = B: never a pivot
            oc_m[i] = ok ? idx % CS : 0;
        }
    }
    // U12 = L11^{-1} A12 of window Wx (rows 0..B-1, columns B..KB-1), a
    // column per lane of wave 0; L11 and the column are read before the
    // substitution starts
    auto u12 = [&](T *Wx) {
        for (int c = B + lane; c < KB; c += 64) {
            T u[B], l11[B][B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                u[t] = Wx[t * WP + c];
#pragma unroll
                for (int s2 = 0; s2 < t; ++s2) l11[t][s2] = Wx[t * WP + s2];
            }
#pragma unroll
            for (int t = 1; t < B; ++t)
#pragma unroll
                for (int s2 = 0; s2 < t; ++s2) u[t] = fma(-l11[t][s2], u[s2], u[t]);
#pragma unroll
            for (int t = 0; t < B; ++t) Wx[t * WP + c] = u[t];
        }
    };
    if (wave == 0) {                                  // panel 0
        T pv[RPL][B];
#pragma unroll
        for (int x = 0; x < RPL; ++x) {
            const int rr = lane + 64 * x;
#pragma unroll
            for (int t = 0; t < B; ++t) pv[x][t] = rr < KB ? win0[rr * WP + t] : T(0);
        }
        factor_panel(pv, (int)min((int64_t)B, nb), uiw);
#pragma unroll
        for (int x = 0; x < RPL; ++x) {
            const int rr = lane + 64 * x;
            if (rr < KB)
#pragma unroll
                for (int t = 0; t < B; ++t) win0[rr * WP + t] = pv[x][t];
        }
        u12(win0);
    }
    __syncthreads();
    // Loop invariant: the panel columns 0..B-1 of the current window are
    // factored.  During the Schur update of panel p (waves 1..), wave 0 forms
    // the next panel's columns of the next window first and factors them
    // (look-ahead), so the panel factorization overlaps the update.
    for (int64_t pnl = 0; pnl < npanel; ++pnl) {
        const int64_t j0 = pnl * B;
        T *W = win0 + (pnl & 1) * KB * WP;            // current window
        T *Wn = win0 + ((pnl + 1) & 1) * KB * WP;     // next window
        const int64_t e0 = j0;                        // entering indices of this panel
        if ((e0 % S) == 0) {
            // the next chunk's loads go out right after this chunk's commit,
            // before this panel's output stores: a wait for the loads then
            // does not also wait for fresh stores
            commit(e0 / S);
            prefetch(e0 / S + 1);
            __syncthreads();                  // the stage is read in 3L
        }
        const int nact = (int)min((int64_t)B, nb - j0);   // pivots in this panel
        const T *stg = stage + (((e0) / S) & 1) * stage_sz + S;

        // 3L. the next window's first B columns and first B rows, by all
        // threads (U12 of this panel was formed with its factorization)
        if (pnl + 1 < npanel) {
            const int pofs = (int)((pnl * B) % S);
#pragma unroll
            for (int i = 0; i < NIL; ++i) {
                if (il_dst[i] < 0) continue;
                T v;
                if (il_row[i] >= 0) {
                    // all operands are read before the first FMA (the
                    // scheduler would otherwise wait on each read in turn)
                    const int ro = il_row[i], co = il_col[i];
                    T lr[B], uc[B];
                    v = W[ro + co];
#pragma unroll
                    for (int t = 0; t < B; ++t) {
                        lr[t] = W[ro + t];
                        uc[t] = W[t * WP + co];
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int t = 0; t < B; ++t) v = fma(-lr[t], uc[t], v);
                } else {
                    v = stg[-1 - il_row[i] - S + pofs];
                }
                Wn[il_dst[i]] = v;
            }
        }
        __syncthreads();
        if (wave == 0) {
            // factorization of the next panel, in registers
            if (pnl + 1 < npanel) {
                T pv[RPL][B];
#pragma unroll
                for (int x = 0; x < RPL; ++x) {
                    const int rr = lane + 64 * x;
#pragma unroll
                    for (int t = 0; t < B; ++t) pv[x][t] = rr < KB ? Wn[rr * WP + t] : T(0);
                }
                factor_panel(pv, (int)min((int64_t)B, nb - j0 - B), uiw + ((pnl + 1) & 1) * B);
#pragma unroll
                for (int x = 0; x < RPL; ++x) {
                    const int rr = lane + 64 * x;
                    if (rr < KB)
#pragma unroll
                        for (int t = 0; t < B; ++t) Wn[rr * WP + t] = pv[x][t];
                }
                u12(Wn);       // rows 0..B-1 of Wn were formed in 3L
            }
        } else {
            const int wr = wave - 1, NR = NW - 1, tr = tid - 64, NTR = NT - 64;
            // 3a. Schur update of the other entries into the next window:
            // Wn[r-B][c-B] = W[r][c] - L21 U12 for window rows and columns
            // >= 2B (rows four at a time, so the LDS reads of four rows are
            // in flight together)
            for (int cb = B + lane; cb < k; cb += 64) {
                const int c = B + cb;
                T uc[B];
#pragma unroll
                for (int t = 0; t < B; ++t) uc[t] = W[t * WP + c];
                int rb = B + wr;                        // rows < B: formed in 3L
                for (; rb + 3 * NR < k; rb += 4 * NR) {
                    T v[4], lr[4][B];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = B + rb + q * NR;
                        v[q] = W[r * WP + c];
#pragma unroll
                        for (int t = 0; t < B; ++t) lr[q][t] = W[r * WP + t];
                    }
                    __builtin_amdgcn_sched_barrier(0);      // reads first, as above
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int t = 0; t < B; ++t) v[q] = fma(-lr[q][t], uc[t], v[q]);
#pragma unroll
                    for (int q = 0; q < 4; ++q) Wn[(rb + q * NR) * WP + cb] = v[q];
                }
                for (; rb < k; rb += NR) {
                    const int r = B + rb;
                    T v = W[r * WP + c], lr[B];
#pragma unroll
                    for (int t = 0; t < B; ++t) lr[t] = W[r * WP + t];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int t = 0; t < B; ++t) v = fma(-lr[t], uc[t], v);
                    Wn[rb * WP + cb] = v;
                }
            }
            // 3b. entering entries of the next window outside its first B
            // columns and rows (items fixed per thread, set up before the loop)
            const int pofs = (int)((pnl * B) % S);
#pragma unroll
            for (int i = 0; i < NIB; ++i)
                if (eb_dst[i] >= 0) Wn[eb_dst[i]] = stg[eb_src[i] + pofs];
            // 3c. outputs of the panel's pivots: L column and U row of j = j0+t
#pragma unroll
            for (int i = 0; i < NIC; ++i) {
                const int t = oc_t[i], m = oc_m[i];
                if (t >= nact) continue;
                const int64_t j = j0 + t;
                const T piv = W[t * WP + t];
                const T lv = m == 0 ? T(1) : W[(t + m) * WP + t];
                const T uv = m == 0 ? uiw[(pnl & 1) * B + t] : W[t * WP + t + m];
                if (!ul) {
                    const bool in = j + m < nb;
                    a.Lc[(s0 + j) * CP + m] = lv;
                    if (in) a.Uc[(s0 + j + m) * CP + m] = uv;
                    if (a.Ur) a.Ur[(s0 + j) * CP + m] = in ? uv : T(0);
                    if (a.Lr && in) a.Lr[(s0 + j + m) * CP + m] = lv;
                } else if (a.corner && j >= nb - k && j + m < nb) {
                    const int64_t b0 = j - (nb - k);
                    T *cn = a.corner + (int64_t)blk * k * k;
                    if (m >= 1) cn[(b0 + m) * k + b0] = lv;
                    cn[b0 * k + b0 + m] = m == 0 ? piv : uv;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && nboost) atomicAdd(&a.status[0], nboost);
    if (tid == 0 && zero_piv) a.status[1] = 1;
}

constexpr size_t kLuBlkStaticLds = 64;   // bytes of static LDS in k_banded_lu_blk (tau_sh), rounded up

template <typename T, int B, int S, int NT, int RPL>
static hipError_t launch_lu_blk(const LuArgs<T> &a, hipStream_t s)
{
    const int k = a.pt.k, KB = k + B;
    const size_t lds = (2 * (size_t)KB * (KB + 1) + 2 * (size_t)(2 * k + 3) * S +
                        2 * (size_t)B) * sizeof(T);
    if (lds + kLuBlkStaticLds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_banded_lu_blk<T, B, S, NT, RPL>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid(a.with_ul ? 2 * a.pt.p : a.pt.p);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <typename T, int WC, int S, int NT>
static hipError_t launch_lu_cfg(const LuArgs<T> &a, hipStream_t s)
{
    const size_t lds = (2 * (size_t)(2 * a.pt.k + 3) * S + (size_t)S * 2 * (a.pt.k + 1)) * sizeof(T);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_banded_lu<T, WC, S, NT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid(a.with_ul ? 2 * a.pt.p : a.pt.p);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, a);
    return hipGetLastError();
}

// LDS of the blocked kernel (two windows, two stage buffers, the reciprocals);
// the static tau_sh takes some of the CU's LDS beside it
static size_t lu_blk_lds(int k, int b, int s, size_t szt)
{
    const size_t kb = (size_t)k + b;
    return (2 * kb * (kb + 1) + 2 * (size_t)(2 * k + 3) * s + 2 * (size_t)b) * szt +
           kLuBlkStaticLds;
}

template <>
hipError_t launch_banded_lu<double>(const LuArgs<double> &a, hipStream_t s)
{
    const int k = a.pt.k;
    // blocked kernel: panel width 8 (the fastest measured at K = 10..50), or 4,
    // with K + B <= 64 (one panel row per lane), then two panel rows per lane
    // while the window fits the LDS with stage chunks of 16 (K <= 78)
    if (k + 8 <= 64) return launch_lu_blk<double, 8, 32, 512, 1>(a, s);
    if (k + 4 <= 64) return launch_lu_blk<double, 4, 32, 512, 1>(a, s);
    if (k + 8 <= 128 && lu_blk_lds(k, 8, 16, sizeof(double)) <= kMaxLds)
        return launch_lu_blk<double, 8, 16, 512, 2>(a, s);
    if (k < 64 && lu_mfma_supported(k, false)) return launch_lu_mfma<double>(a, s);
    // matrix-core kernel where its register window fits without spilling
    // (K <= 96), the register ring up to K = 127, then the matrix-core kernel
    // again (its larger windows spill part of the registers)
    if (k >= 64 && k <= 96) return launch_lu_mfma<double>(a, s);
    if (k >= 128 && lu_mfma_supported(k, false)) return launch_lu_mfma<double>(a, s);
    if (k < 16) return launch_lu_cfg<double, 16, 16, 256>(a, s);
    if (k < 32) return launch_lu_cfg<double, 32, 32, 256>(a, s);
    if (k < 64) return launch_lu_cfg<double, 64, 32, 256>(a, s);
    if (k < 128) return launch_lu_cfg<double, 128, 16, 1024>(a, s);
    return launch_lu_wide(a, a.wide, s);      // K > 160
}

template <>
hipError_t launch_banded_lu<float>(const LuArgs<float> &a, hipStream_t s)
{
    const int k = a.pt.k;
    // blocked kernel: panel width 8 (the fastest measured at K = 10..50), or 4,
    // with K + B <= 64 (one panel row per lane), then two panel rows per lane
    // while the double-buffered window fits the LDS (K <= 104)
    if (k + 8 <= 64) return launch_lu_blk<float, 8, 32, 512, 1>(a, s);
    if (k + 4 <= 64) return launch_lu_blk<float, 4, 32, 512, 1>(a, s);
    if (k + 8 <= 128 && lu_blk_lds(k, 8, 32, sizeof(float)) <= kMaxLds)
        return launch_lu_blk<float, 8, 32, 512, 2>(a, s);
    if (k < 64 && lu_mfma_supported(k, true)) return launch_lu_mfma<float>(a, s);
    if (k >= 64 && lu_mfma_supported(k, true)) return launch_lu_mfma<float>(a, s);
    if (k < 16) return launch_lu_cfg<float, 16, 16, 256>(a, s);
    if (k < 32) return launch_lu_cfg<float, 32, 32, 256>(a, s);
    if (k < 64) return launch_lu_cfg<float, 64, 32, 256>(a, s);
    if (k < 128) return launch_lu_cfg<float, 128, 32, 1024>(a, s);
    return launch_lu_cfg<float, 256, 16, 1024>(a, s);
}

}  // namespace sap
