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

namespace sap {

// ---------------------------------------------------------------- norms

// partial[blk][chunk] = max |a_rc| over the columns of one 256-column chunk
// of diagonal block blk (rows restricted to the block).
__global__ __launch_bounds__(256) void k_block_norm(const double *__restrict__ band,
                                                    Partition pt,
                                                    double *__restrict__ partial,
                                                    int nchunk)
{
    const int blk = blockIdx.y;
    const int64_t s0 = pt.starts[blk];
    const int64_t nb = pt.starts[blk + 1] - s0;
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double m = 0.0;
    if (x < nb) {
        const int64_t c = s0 + x;
        for (int q = 0; q <= 2 * pt.k; ++q) {
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
                             int nchunk, hipStream_t s)
{
    dim3 grid(nchunk, pt.p);
    hipLaunchKernelGGL(k_block_norm, grid, dim3(256), 0, s, band, pt, partial, nchunk);
    return hipGetLastError();
}

// ------------------------------------------------------------------- LU

// Entry (r, c) of the block as seen by the LU (ul = 0) or by the LU of the
// reversed block (ul = 1); 0 outside the block or the band.
__device__ __forceinline__ double block_entry(const double *__restrict__ band, int64_t n,
                                              int k, int64_t s0, int64_t nb, int ul,
                                              int64_t r, int64_t c)
{
    const int64_t d = r - c;
    if (r < 0 || c < 0 || r >= nb || c >= nb || d > k || d < -k) return 0.0;
    const int64_t q = ul ? (k - d) : (k + d);
    const int64_t col = ul ? (s0 + nb - 1 - c) : (s0 + c);
    return band[q * n + col];
}

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
                a.Uc[(s0 + c) * CS + m] = T(0);
                if (a.Lr) a.Lr[(s0 + c) * CS + m] = T(0);
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
    T pre[PR];
    auto prefetch = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            const int q = f / S, ss = f % S;              // S is a power of two
            const int delta = q - k;
            const int64_t m = WC + t * S + ss;
            T v = T(0);
            if (f < W2 * S && m < nb) {  // m > K >= |delta|: other index >= 0
                const int64_t base = (int64_t)(ul ? (k - delta) : (k + delta)) * n;
                const int64_t col = ul ? (s0 + nb - 1 - m + (delta > 0 ? delta : 0))
                                       : (s0 + m - (delta > 0 ? delta : 0));
                v = (T)a.band[base + col];
            }
            pre[i] = v;
        }
    };
    auto commit = [&](int64_t t) {
        T *dst = stage + (t & 1) * stage_sz + S;
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int f = tid + NT * i;
            if (f < W2 * S) dst[f] = pre[i];
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
            a.Lc[(s0 + j) * CS + m] = lv;
            if (in) a.Uc[(s0 + j + m) * CS + m] = uv;
            if (a.Ur) a.Ur[(s0 + j) * CS + m] = in ? uv : T(0);
            if (a.Lr && in) a.Lr[(s0 + j + m) * CS + m] = lv;
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

template <typename T, int WC, int S, int NT>
static hipError_t launch_lu_cfg(const LuArgs<T> &a, hipStream_t s)
{
    const size_t lds = (2 * (size_t)(2 * a.pt.k + 3) * S + (size_t)S * 2 * (a.pt.k + 1)) * sizeof(T);
    auto kern = k_banded_lu<T, WC, S, NT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid(a.with_ul ? 2 * a.pt.p : a.pt.p);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, a);
    return hipGetLastError();
}

template <>
hipError_t launch_banded_lu<double>(const LuArgs<double> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (k < 16) return launch_lu_cfg<double, 16, 16, 256>(a, s);
    if (k < 32) return launch_lu_cfg<double, 32, 32, 256>(a, s);
    if (k < 64) return launch_lu_cfg<double, 64, 32, 256>(a, s);
    if (k < 128) return launch_lu_cfg<double, 128, 16, 1024>(a, s);
    return hipErrorInvalidValue;   // FP64 window for K >= 128 exceeds the VGPR budget
}

template <>
hipError_t launch_banded_lu<float>(const LuArgs<float> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (k < 16) return launch_lu_cfg<float, 16, 16, 256>(a, s);
    if (k < 32) return launch_lu_cfg<float, 32, 32, 256>(a, s);
    if (k < 64) return launch_lu_cfg<float, 64, 32, 256>(a, s);
    if (k < 128) return launch_lu_cfg<float, 128, 32, 1024>(a, s);
    return launch_lu_cfg<float, 256, 16, 1024>(a, s);
}

}  // namespace sap
