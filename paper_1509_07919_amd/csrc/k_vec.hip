// Bandwidth-bound kernels of the solve: banded SpMV (and A^T), the band of
// the gradient -lambda x^T, the SaP-C interface correction, and the fused
// vector updates + dot products of BiCGStab(2).
#include "sap_internal.h"

namespace sap {

// --------------------------------------------------------------- SpMV
// y_r = sum_q band[q*n + c] v_c with c = r + K - q (A v), or
// y_c = sum_q band[q*n + c] v_{c+q-K} (A^T v).  A workgroup takes 64
// outputs: lane l of wave w owns output r0 + l and the diagonals q = w
// (mod 4), so for a fixed q a wave reads one coalesced 512-byte run of the
// band, and four times as many waves as outputs / 256 keep enough loads in
// flight for HBM.  The v tile [r0-K, r0+64+K) is staged once in LDS and the
// four partial sums are added in LDS.  Optional residual form b - A v.
constexpr int kSpmvRows = 64;
// NR right-hand sides at once (multi-RHS solves): every band entry read
// serves NR columns; v columns c0 .. c0+NR-1 of a column-major block with
// leading dimension ld (columns past m are skipped).
template <int NR>
__global__ __launch_bounds__(256) void k_spmv(const double *__restrict__ band, int64_t n,
                                              int k, const double *__restrict__ v,
                                              const double *__restrict__ b,
                                              double *__restrict__ y, int trans, int64_t ld,
                                              int m)
{
    __shared__ double vt[NR][kSpmvRows + 2 * kMaxK];
    __shared__ double part[3][NR][kSpmvRows];
    const int c0 = (int)blockIdx.y * NR;
    const int nc = min(NR, m - c0);
    const int64_t r0 = (int64_t)blockIdx.x * kSpmvRows;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j >= nc) break;
        const double *vj = v + (int64_t)(c0 + j) * ld;
        for (int i = tid; i < kSpmvRows + 2 * k; i += 256) {
            const int64_t g = r0 - k + i;
            vt[j][i] = (g >= 0 && g < n) ? vj[g] : 0.0;
        }
    }
    __syncthreads();
    const int64_t r = r0 + lane;
    const int w = 2 * k + 1;
    double acc0[NR], acc1[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc0[j] = acc1[j] = 0.0;
    if (r < n) {
        if (!trans) {
            // a[r][c] at band[(k + r - c)*n + c]; c = r + k - q in [0, n)
            const int qlo = (int)max((int64_t)0, r + k - (n - 1));
            const int qhi = (int)min((int64_t)(w - 1), r + k);
            int q = qlo + ((wave - qlo) & 3);
            for (; q + 4 <= qhi; q += 8) {
                const double a0 = band[(int64_t)q * n + (r + k - q)];
                const double a1 = band[(int64_t)(q + 4) * n + (r + k - q - 4)];
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    acc0[j] = fma(a0, vt[j][lane + 2 * k - q], acc0[j]);
                    acc1[j] = fma(a1, vt[j][lane + 2 * k - q - 4], acc1[j]);
                }
            }
            if (q <= qhi) {
                const double a0 = band[(int64_t)q * n + (r + k - q)];
#pragma unroll
                for (int j = 0; j < NR; ++j) acc0[j] = fma(a0, vt[j][lane + 2 * k - q], acc0[j]);
            }
        } else {
            // a[rr][r] at band[q*n + r] with rr = r + q - k in [0, n)
            const int qlo = (int)max((int64_t)0, (int64_t)k - r);
            const int qhi = (int)min((int64_t)(w - 1), n - 1 - r + k);
            int q = qlo + ((wave - qlo) & 3);
            for (; q + 4 <= qhi; q += 8) {
                const double a0 = band[(int64_t)q * n + r];
                const double a1 = band[(int64_t)(q + 4) * n + r];
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    acc0[j] = fma(a0, vt[j][lane + q], acc0[j]);
                    acc1[j] = fma(a1, vt[j][lane + q + 4], acc1[j]);
                }
            }
            if (q <= qhi) {
                const double a0 = band[(int64_t)q * n + r];
#pragma unroll
                for (int j = 0; j < NR; ++j) acc0[j] = fma(a0, vt[j][lane + q], acc0[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (wave > 0) part[wave - 1][j][lane] = acc0[j] + acc1[j];
    __syncthreads();
    if (wave == 0 && r < n) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (j >= nc) break;
            const double acc = acc0[j] + acc1[j];
            const double tot = (acc + part[0][j][lane]) + (part[1][j][lane] + part[2][j][lane]);
            const int64_t o = (int64_t)(c0 + j) * ld + r;
            y[o] = b ? b[o] - tot : tot;
        }
    }
}

hipError_t launch_spmv(const double *band, int64_t n, int k, const double *v,
                       const double *b, double *y, int trans, hipStream_t s)
{
    const int64_t nblk = (n + kSpmvRows - 1) / kSpmvRows;
    hipLaunchKernelGGL(k_spmv<1>, dim3((unsigned)nblk), dim3(256), 0, s, band, n, k, v, b, y,
                       trans, n, 1);
    return hipGetLastError();
}

hipError_t launch_spmv_multi(const double *band, int64_t n, int k, const double *v,
                             const double *b, double *y, int trans, int m, hipStream_t s)
{
    if (m < 1) return hipErrorInvalidValue;
    if (m == 1) return launch_spmv(band, n, k, v, b, y, trans, s);
    const int64_t nblk = (n + kSpmvRows - 1) / kSpmvRows;
    hipLaunchKernelGGL(k_spmv<kMultiRhs>, dim3((unsigned)nblk, (unsigned)((m + kMultiRhs - 1) / kMultiRhs)),
                       dim3(256), 0, s, band, n, k, v, b, y, trans, n, m);
    return hipGetLastError();
}

// g = band(-lambda x^T): diagonal q of the band (row = column + q - K) is
// one row of the grid, its columns spread over blockIdx.x, so no thread
// divides an index; lambda and x (N doubles each) are re-read from cache by
// every diagonal.
__global__ __launch_bounds__(256) void k_band_grad(int64_t n, int k,
                                                   const double *__restrict__ lam,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ g)
{
    const int64_t d = (int64_t)blockIdx.y - k;
    double *gq = g + (int64_t)blockIdx.y * n;
    // four columns per thread, 256 apart (each store instruction of a wave
    // still covers 64 consecutive slots)
    for (int64_t c0 = (int64_t)blockIdx.x * 1024 + threadIdx.x; c0 < n; c0 += (int64_t)gridDim.x * 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t c = c0 + 256 * u;
            const int64_t r = c + d;
            if (c < n) gq[c] = (r >= 0 && r < n) ? -lam[r] * x[c] : 0.0;
        }
    }
}

hipError_t launch_band_grad(int64_t n, int k, const double *lam, const double *x, double *g,
                            hipStream_t s)
{
    const int64_t nblk = min((n + 1023) / 1024, (int64_t)4096);
    hipLaunchKernelGGL(k_band_grad, dim3((unsigned)nblk, (unsigned)(2 * k + 1)), dim3(256), 0, s,
                       n, k, lam, x, g);
    return hipGetLastError();
}

// ------------------------------------------------------ SaP-C correction
// Interface i couples blocks i and i+1 (s1 = first row of block i+1).
// Forward (eq:solveTopBottom and purification), from g = D^{-1} r:
//   y = Rbar^{-1}(g^(t)_{i+1} - W g^(b)_i),  z = g^(b)_i - V y
//   dbot_i = -B_i y,  dtop_{i+1} = -C_{i+1} z     (added to r before D^{-1})
// Transposed, from h = D^{-T} s:
//   ybar = -B^T h^(b)_i,  zbar = -C^T h^(t)_{i+1},  tbar = Rbar^{-T}(ybar - V^T zbar)
//   dtop_{i+1} = tbar,    dbot_i = zbar - W^T tbar  (added to s before D^{-T})
template <typename T>
__global__ __launch_bounds__(256) void k_correction(CorrArgs<T> a)
{
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int64_t s1 = a.pt.starts[i + 1];
    const int64_t kk = (int64_t)k * k;
    const T *B = a.B + i * kk, *C = a.C + i * kk, *V = a.V + i * kk, *W = a.W + i * kk;
    const T *RI = a.Rinv + i * kk;
    __shared__ T vb[kMaxK], vt[kMaxK], w1[kMaxK], w2[kMaxK], w3[kMaxK];
    const int t = threadIdx.x;
    const int64_t col = blockIdx.y;             // right-hand side
    const T *g = a.g + col * a.ldg;
    if (t < k) {
        vb[t] = g[s1 - k + t];
        vt[t] = g[s1 + t];
    }
    __syncthreads();
    T *dbot = a.dbot + (col * a.pt.p + i) * k;       // bottom rows of block i
    T *dtop = a.dtop + (col * a.pt.p + i + 1) * k;   // top rows of block i+1
    if (!a.trans) {
        if (t < k) {
            T s = vt[t];
            for (int c = 0; c < k; ++c) s = fma(-W[t * k + c], vb[c], s);
            w1[t] = s;
        }
        __syncthreads();
        if (t < k) {
            T s = T(0);
            for (int c = 0; c < k; ++c) s = fma(RI[t * k + c], w1[c], s);
            w2[t] = s;                                   // y
        }
        __syncthreads();
        if (t < k) {
            T s = vb[t];
            for (int c = 0; c < k; ++c) s = fma(-V[t * k + c], w2[c], s);
            w3[t] = s;                                   // z
        }
        __syncthreads();
        if (t < k) {
            T sb = T(0), st = T(0);
            for (int c = 0; c < k; ++c) {
                sb = fma(B[t * k + c], w2[c], sb);
                st = fma(C[t * k + c], w3[c], st);
            }
            dbot[t] = -sb;
            dtop[t] = -st;
        }
    } else {
        if (t < k) {
            T sy = T(0), sz = T(0);
            for (int c = 0; c < k; ++c) {
                sy = fma(B[c * k + t], vb[c], sy);
                sz = fma(C[c * k + t], vt[c], sz);
            }
            w1[t] = -sy;                                 // ybar
            w2[t] = -sz;                                 // zbar
        }
        __syncthreads();
        if (t < k) {
            T s = w1[t];
            for (int c = 0; c < k; ++c) s = fma(-V[c * k + t], w2[c], s);
            w3[t] = s;                                   // ybar - V^T zbar
        }
        __syncthreads();
        if (t < k) {
            T s = T(0);
            for (int c = 0; c < k; ++c) s = fma(RI[c * k + t], w3[c], s);
            w1[t] = s;                                   // tbar
        }
        __syncthreads();
        if (t < k) {
            T s = w2[t];
            for (int c = 0; c < k; ++c) s = fma(-W[c * k + t], w1[c], s);
            dbot[t] = s;
            dtop[t] = w1[t];
        }
    }
}

// The same correction with the interface's five K x K matrices (W, Rinv, V,
// B, C) staged in LDS by one coalesced pass, so their loads overlap, and each
// mat-vec spread over four threads per row (partial sums over c = q mod 4,
// added with two lane exchanges).  Used when they fit in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_correction_lds(CorrArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;
    const int k = a.pt.k;
    const int kk = k * k;
    const int64_t s1 = a.pt.starts[i + 1];
    const int64_t ikk = (int64_t)i * kk;
    T *sm = reinterpret_cast<T *>(smem_raw);
    T *Ws = sm, *Rs = sm + kk, *Vs = sm + 2 * kk, *Bs = sm + 3 * kk, *Cs = sm + 4 * kk;
    T *vb = sm + 5 * kk, *vt = vb + k, *w1 = vt + k, *w2 = w1 + k, *w3 = w2 + k;
    const int t = threadIdx.x;
    for (int e = t; e < kk; e += 256) {
        const T w = a.W[ikk + e], r = a.Rinv[ikk + e], v = a.V[ikk + e];
        const T b = a.B[ikk + e], c = a.C[ikk + e];
        Ws[e] = w; Rs[e] = r; Vs[e] = v; Bs[e] = b; Cs[e] = c;
    }
    const int64_t col = blockIdx.y;             // right-hand side
    const T *g = a.g + col * a.ldg;
    if (t < k) {
        vb[t] = g[s1 - k + t];
        vt[t] = g[s1 + t];
    }
    __syncthreads();
    const int r = t >> 2, q = t & 3;
    const bool act = r < k;
    // sum_c M[r][c] x[c] (tr: M[c][r]) over this thread's c, then over the 4
    auto mv = [&](const T *M, bool tr, const T *x) {
        T s = T(0);
        if (act)
            for (int c = q; c < k; c += 4) s = fma(tr ? M[c * k + r] : M[r * k + c], x[c], s);
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        return s;
    };
    T *dbot = a.dbot + (col * a.pt.p + i) * k;       // bottom rows of block i
    T *dtop = a.dtop + (col * a.pt.p + i + 1) * k;   // top rows of block i+1
    const bool lead = act && q == 0;
    if (!a.trans) {
        T s = mv(Ws, false, vb);
        if (lead) w1[r] = vt[r] - s;
        __syncthreads();
        s = mv(Rs, false, w1);
        if (lead) w2[r] = s;                                 // y
        __syncthreads();
        s = mv(Vs, false, w2);
        if (lead) w3[r] = vb[r] - s;                         // z
        __syncthreads();
        const T sb = mv(Bs, false, w2), st = mv(Cs, false, w3);
        if (lead) {
            dbot[r] = -sb;
            dtop[r] = -st;
        }
    } else {
        const T sy = mv(Bs, true, vb), sz = mv(Cs, true, vt);
        if (lead) {
            w1[r] = -sy;                                     // ybar
            w2[r] = -sz;                                     // zbar
        }
        __syncthreads();
        T s = mv(Vs, true, w2);
        if (lead) w3[r] = w1[r] - s;                         // ybar - V^T zbar
        __syncthreads();
        s = mv(Rs, true, w3);
        if (lead) w1[r] = s;                                 // tbar
        __syncthreads();
        s = mv(Ws, true, w1);
        if (lead) {
            dbot[r] = w2[r] - s;
            dtop[r] = w1[r];
        }
    }
}

template <typename T>
hipError_t launch_correction(const CorrArgs<T> &a0, hipStream_t s)
{
    CorrArgs<T> a = a0;              // one right-hand side unless stated
    if (a.m < 1) a.m = 1;
    if (a.pt.p < 2 || a.pt.k == 0) return hipSuccess;
    const size_t kk = (size_t)a.pt.k * a.pt.k;
    const size_t lds = (5 * kk + 5 * (size_t)a.pt.k) * sizeof(T);
    if (lds <= kMaxLds && a.pt.k <= 64) {
        auto kern = k_correction_lds<T>;
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(a.pt.p - 1, a.m), dim3(256), lds, s, a);
    } else {
        hipLaunchKernelGGL(k_correction<T>, dim3(a.pt.p - 1, a.m), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}
template hipError_t launch_correction<float>(const CorrArgs<float> &, hipStream_t);
template hipError_t launch_correction<double>(const CorrArgs<double> &, hipStream_t);

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Scalar recurrences of BiCGStab(2) (Sleijpen-Fokkema), run by one thread
// once the dots d[] of a launch are complete.
__device__ void scalar_op(int op, const double *d, double *sc, double *host)
{
    auto brk = [&](double code) {
        if (sc[S_BREAK] == 0.0) sc[S_BREAK] = code;
    };
    auto prep_j0 = [&](double rho1) {     // rho0 = -omega rho0; beta; rho0 = rho1
        sc[S_RHO0] = -sc[S_OMEGA] * sc[S_RHO0];
        if (sc[S_RHO0] == 0.0) brk(1.0);
        sc[S_BETA] = sc[S_ALPHA] * rho1 / sc[S_RHO0];
        sc[S_RHO0] = rho1;
    };
    bool publish = false;
    switch (op) {
    case OP_INIT:
        sc[S_RHO0] = 1.0; sc[S_ALPHA] = 0.0; sc[S_OMEGA] = 1.0; sc[S_BREAK] = 0.0;
        sc[S_NRM2] = d[1]; publish = true;
        prep_j0(d[0]);
        break;
    case OP_GAMMA:
        sc[S_GAMMA] = d[0];
        if (d[0] == 0.0) brk(2.0);
        sc[S_ALPHA] = sc[S_RHO0] / d[0];
        break;
    case OP_TRUE:
        if (host) host[H_TRUE] = d[0];
        break;
    case OP_SPEC:
        if (host) host[H_SPEC] = d[0];
        break;
    case OP_BNORM:
        if (host) host[H_BNORM] = d[0];
        break;
    case OP_EXIT:
    case OP_NORM:
        sc[S_NRM2] = d[0]; publish = true;
        break;
    case OP_RHO:
        if (sc[S_RHO0] == 0.0) brk(1.0);
        sc[S_BETA] = sc[S_ALPHA] * d[0] / sc[S_RHO0];
        sc[S_RHO0] = d[0];
        break;
    case OP_MR1:
        sc[S_SIGMA1] = d[0];
        if (d[0] == 0.0) brk(3.0);
        sc[S_GP1] = d[1] / d[0];
        sc[S_TAU12] = d[2] / d[0];
        break;
    case OP_MR2: {
        sc[S_SIGMA2] = d[0];
        if (d[0] == 0.0) brk(3.0);
        const double gp2 = d[1] / d[0];
        sc[S_GP2] = gp2;
        sc[S_G2] = gp2;
        sc[S_OMEGA] = gp2;
        sc[S_G1] = sc[S_GP1] - sc[S_TAU12] * gp2;
        sc[S_GPP1] = gp2;
        break;
    }
    case OP_FINAL:
        sc[S_NRM2] = d[0]; publish = true;
        prep_j0(d[1]);
        break;
    case OP_CG_INIT:
        sc[S_BREAK] = 0.0;
        sc[S_RHO0] = d[0];
        sc[S_NRM2] = d[1]; publish = true;
        break;
    case OP_CG_ALPHA:
        if (!(d[0] > 0.0)) brk(4.0);
        sc[S_ALPHA] = sc[S_RHO0] / d[0];
        break;
    case OP_CG_BETA:
        if (sc[S_RHO0] == 0.0) brk(1.0);
        sc[S_BETA] = d[0] / sc[S_RHO0];
        sc[S_RHO0] = d[0];
        break;
    default:
        break;
    }
    if (host) {
        if (publish) host[H_NRM2] = sc[S_NRM2];
        if (op == OP_INIT || op == OP_CG_INIT) host[H_NRM0] = sc[S_NRM2];
        host[H_BREAK] = sc[S_BREAK];
    }
}

// Block-reduce up to three per-thread sums and store this block's partials.
// Multi-RHS form: column col of the vectors (ld apart) has its own partials,
// scalars and host slots; frozen columns (bit col of a.frozen) are skipped.
__device__ __forceinline__ bool col_frozen(const DotArgs &a, int col)
{
    return col < 64 && ((a.frozen >> col) & 1ull);
}

__device__ void finish_dots(const DotArgs &a, double l0, double l1, double l2)
{
    __shared__ double red[3][4];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const double s0 = wave_sum(l0), s1 = wave_sum(l1), s2 = wave_sum(l2);
    if (lane == 0) { red[0][wid] = s0; red[1][wid] = s1; red[2][wid] = s2; }
    __syncthreads();
    if (tid == 0)
        for (int d = 0; d < 3; ++d)
            a.partial[((int64_t)blockIdx.y * kDotBlocks + blockIdx.x) * 3 + d] =
                (red[d][0] + red[d][1]) + (red[d][2] + red[d][3]);
}

// One workgroup combines the kDotBlocks partials of the preceding launch in a
// fixed order (so the result is bitwise reproducible) and runs the scalar
// recurrence.  The kernel boundary makes the partials visible, so the
// producing blocks need no fence or ticket.
__global__ __launch_bounds__(256) void k_dots_final(DotArgs a)
{
    __shared__ double tot[3][256];
    const int tid = threadIdx.x;
    const int col = blockIdx.x;
    if (col_frozen(a, col)) return;
    const double *part = a.partial + (int64_t)col * kDotBlocks * 3;
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int b = tid; b < kDotBlocks; b += 256) s += part[b * 3 + d];
        tot[d][tid] = s;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int d = 0; d < 3; ++d) tot[d][tid] += tot[d][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const double dd[3] = {tot[0][0], tot[1][0], tot[2][0]};
        scalar_op(a.op, dd, a.sc + (int64_t)col * kScalars,
                  a.host ? a.host + (int64_t)col * kHostSlots : nullptr);
        if (a.status && a.host && col == 0) {
            a.host[H_NBOOST] = (double)a.status[0];
            a.host[H_SING] = (double)a.status[1];
        }
        __threadfence_system();
    }
}

__global__ __launch_bounds__(256) void k_dots(DotArgs a)
{
    const int col = blockIdx.y;
    if (col_frozen(a, col)) return;
    const int64_t off = (int64_t)col * a.ld;
    double l[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * 256) {
        for (int d = 0; d < 3; ++d)
            if (d < a.nd) l[d] = fma(a.x[d][off + i], a.y[d][off + i], l[d]);
    }
    finish_dots(a, l[0], l[1], l[2]);
}

hipError_t launch_dots(const DotArgs &a0, hipStream_t s)
{
    DotArgs a = a0;
    if (a.m < 1) a.m = 1;
    hipLaunchKernelGGL(k_dots, dim3(kDotBlocks, a.m), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_dots_final, dim3(a.m), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_update(UpdArgs a)
{
    const int col = blockIdx.y;
    if (col_frozen(a.dots, col)) return;
    if (col > 0) {               // column col of every vector, its own scalars
        const int64_t off = (int64_t)col * a.dots.ld;
        for (double **v : {&a.x, &a.r0, &a.r1, &a.r2, &a.u0, &a.u1, &a.u2, &a.rt})
            if (*v) *v += off;
    }
    const double *sc = a.dots.sc + (int64_t)col * kScalars;
    const double beta = sc[S_BETA], alpha = sc[S_ALPHA], tau12 = sc[S_TAU12];
    const double g1 = sc[S_G1], g2 = sc[S_G2], gp1 = sc[S_GP1], gp2 = sc[S_GP2],
                 gpp1 = sc[S_GPP1];
    double l0 = 0.0, l1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * 256) {
        switch (a.kind) {
        case UPD_U0:
            a.u0[i] = a.r0[i] - beta * a.u0[i];
            break;
        case UPD_J0: {
            const double r = a.r0[i] - alpha * a.u1[i];
            a.r0[i] = r;
            a.x[i] += alpha * a.u0[i];
            l0 = fma(r, r, l0);
            break;
        }
        case UPD_U01:
            a.u0[i] = a.r0[i] - beta * a.u0[i];
            a.u1[i] = a.r1[i] - beta * a.u1[i];
            break;
        case UPD_J1: {
            const double r = a.r0[i] - alpha * a.u1[i];
            a.r0[i] = r;
            a.r1[i] -= alpha * a.u2[i];
            a.x[i] += alpha * a.u0[i];
            l0 = fma(r, r, l0);
            break;
        }
        case UPD_MR2: {
            const double r2 = a.r2[i] - tau12 * a.r1[i];
            a.r2[i] = r2;
            l0 = fma(r2, r2, l0);
            l1 = fma(a.r0[i], r2, l1);
            break;
        }
        case UPD_FINAL: {
            const double r0 = a.r0[i], r1 = a.r1[i];
            a.x[i] += g1 * r0 + gpp1 * r1;
            const double rn = r0 - gp2 * a.r2[i] - gp1 * r1;
            a.r0[i] = rn;
            a.u0[i] = a.u0[i] - g2 * a.u2[i] - g1 * a.u1[i];
            l0 = fma(rn, rn, l0);
            l1 = fma(rn, a.rt[i], l1);
            break;
        }
        case UPD_RESTART: {
            const double r = a.r0[i];
            a.rt[i] = r;
            a.u0[i] = 0.0;
            l0 = fma(r, r, l0);        // (r0, rt) = (r0, r0)
            break;
        }
        case UPD_CG_INIT: {
            const double r = a.r0[i], z = a.r1[i];
            a.u0[i] = z;
            l0 = fma(r, z, l0);
            l1 = fma(r, r, l1);
            break;
        }
        case UPD_CG_XR: {
            a.x[i] += alpha * a.u0[i];
            const double r = a.r0[i] - alpha * a.u1[i];
            a.r0[i] = r;
            l0 = fma(r, r, l0);
            break;
        }
        case UPD_CG_P:
            a.u0[i] = a.r1[i] + beta * a.u0[i];
            break;
        default:
            break;
        }
    }
    if (a.dots.nd == 0) return;
    if (a.kind == UPD_RESTART) l1 = l0;
    // dot order per kind: J0/J1 -> (r0,r0); MR2 -> (r2,r2),(r0,r2);
    // FINAL -> (r0,r0),(r0,rt); RESTART -> (r0,rt),(r0,r0);
    // CG_INIT -> (r,z),(r,r); CG_XR -> (r,r)
    finish_dots(a.dots, l0, l1, 0.0);
}

hipError_t launch_update(const UpdArgs &a0, hipStream_t s)
{
    UpdArgs a = a0;
    if (a.dots.m < 1) a.dots.m = 1;
    hipLaunchKernelGGL(k_update, dim3(kDotBlocks, a.dots.m), dim3(256), 0, s, a);
    if (a.dots.nd > 0) hipLaunchKernelGGL(k_dots_final, dim3(a.dots.m), dim3(256), 0, s, a.dots);
    return hipGetLastError();
}

__global__ void k_fill(double *v, double val, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        v[i] = val;
}

hipError_t launch_fill(double *v, double val, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(kDotBlocks), dim3(256), 0, s, v, val, n);
    return hipGetLastError();
}

// zero `words` 32-bit words (used instead of a memset node, so the callers
// stay capturable into a graph)
__global__ void k_zero32(unsigned *v, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * 256)
        v[i] = 0u;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t words = (int64_t)(bytes / 4);
    if (words == 0) return hipSuccess;
    const int64_t want = (words + 255) / 256;
    const int grid = (int)(want < kDotBlocks ? want : kDotBlocks);
    hipLaunchKernelGGL(k_zero32, dim3(grid), dim3(256), 0, s, static_cast<unsigned *>(p), words);
    return hipGetLastError();
}

// Block boundaries of Sec. 3.1 (first P_r = N - P floor(N/P) blocks one row
// longer), computed on the device so that no host buffer is involved.
__global__ void k_partition_starts(int64_t *starts, int64_t n, int p)
{
    const int64_t q = n / p, pr = n - (int64_t)p * q;
    for (int i = (int)(blockIdx.x * 256 + threadIdx.x); i <= p; i += (int)(gridDim.x * 256))
        starts[i] = (int64_t)i * q + (i < pr ? i : pr);
}

hipError_t launch_partition_starts(int64_t *starts, int64_t n, int p, hipStream_t s)
{
    const int grid = (p + 1 + 255) / 256;
    hipLaunchKernelGGL(k_partition_starts, dim3(grid), dim3(256), 0, s, starts, n, p);
    return hipGetLastError();
}

}  // namespace sap
