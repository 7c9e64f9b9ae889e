// Forward elimination / back substitution with the block factors (the
// block-diagonal solves D g = b of eq:diag-sys, and the purification solves
// of Sec. 2.1), arXiv:1509.07919 Sec. 3.1: each is a chain of N_i dependent
// steps per block.
//
// Every sweep is written in "push" form over a coefficient array F with one
// row of K+1 entries per step (see sap_internal.h):
//     x_j = (v_j - p_j) * F[j][0],        p_{j+-m} += F[j][m] * x_j
// (the kernel keeps acc = -p).
// L (forward, unit), U (backward), U^T (forward) and L^T (backward) differ
// only in the array and the direction.
//
// MI355X design.  One workgroup per block: wave 0 runs the dependent chain,
// waves 1-3 stream the coefficient rows and the input vector of the next
// chunk of S steps from HBM into double-buffered LDS (a contiguous S*(K+1)
// run per chunk).  The pending sums acc_{j+1..j+K} live in wave 0's VGPRs:
// register s, lane l holds the step 64*s + l counted from the start of the
// current 64-step block; KR = 1 + ceil(K/64) registers cover the reach of
// step 63 of the block (63 + K), and the registers shift down by one every
// 64 steps, so register indices stay static for any K <= 255.
// Per step: one FMA for x_j in lane u, a v_readlane broadcast (lane index in
// an SGPR), and one FMA per register in every lane.  Outputs are gathered in a register and
// written 64 at a time, coalesced.
#include "sap_internal.h"

namespace sap {

__device__ __forceinline__ double lane_bcast(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <typename T, int KR, int S, bool FWD, bool DIAG>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a)
{
    static_assert(S % 64 == 0, "chunk must hold whole 64-step blocks");
    static_assert(KR >= 2, "ring must cover 64 + K slots");
    // LDS row pitch: slots 0..K hold a coefficient row, slots K+1..PITCH-1
    // are zero (the last 8 always), so a clamped offset needs no mask
    constexpr int PITCH = 64 * (KR - 1) + 8;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *cst = reinterpret_cast<T *>(smem_raw);         // [2][S][PITCH]
    T *vst = cst + 2 * S * PITCH;                     // [2][S]

    const int k = a.pt.k;
    const int CS = k + 1;
    const int blk = blockIdx.x;
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int64_t nchunks = (nb + S - 1) / S;
    const T *dtop = (a.dtop && blk > 0) ? a.dtop + (int64_t)blk * k : nullptr;
    const T *dbot = (a.dbot && blk < a.pt.p - 1) ? a.dbot + (int64_t)blk * k : nullptr;

    for (int idx = tid; idx < 2 * S * 8; idx += 256)
        cst[(idx >> 3) * PITCH + 64 * (KR - 1) + (idx & 7)] = T(0);

    // row of the block handled at step t
    auto row_of = [&](int64_t t) -> int64_t { return FWD ? t : nb - 1 - t; };

    if (wave != 0) {
        // ------------------------------------------------------ loaders
        // loader wave lw (0..2) stages chunk rows lw, lw+3, ...; lane l loads
        // coefficient slots l, l+64, ... of each row, and the input values of
        // the chunk are spread over all loader threads
        const int lw = wave - 1;
        constexpr int RPW = (S + 2) / 3;              // rows per loader wave
        constexpr int NSEG = KR - 1;                  // 64-slot segments per row
        T pre[RPW * NSEG];
        T vin = T(0);
        auto load = [&](int64_t t) {
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                const int rr = lw + 3 * y;                    // row inside the chunk
                const int64_t st = t * S + rr;
                const bool ok = rr < S && st < nb;
                const T *src = a.F + (s0 + (ok ? row_of(st) : 0)) * CS;
#pragma unroll
                for (int x = 0; x < NSEG; ++x) {
                    const int m = lane + 64 * x;
                    pre[y * NSEG + x] = (ok && m < CS) ? src[m] : T(0);
                }
            }
            const int f = tid - 64;
            vin = T(0);
            if (f < S) {
                const int64_t st = t * S + f;
                if (st < nb) {
                    const int64_t r = row_of(st);
                    if (a.xin) {
                        double x = a.xin[s0 + r];
                        if (dtop && r < k) x += (double)dtop[r];
                        if (dbot && r >= nb - k) x += (double)dbot[r - (nb - k)];
                        vin = (T)x;
                    } else {
                        T x = a.tin[s0 + r];
                        if (dtop && r < k) x += dtop[r];
                        if (dbot && r >= nb - k) x += dbot[r - (nb - k)];
                        vin = x;
                    }
                }
            }
        };
        auto commit = [&](int64_t t) {
            T *c = cst + (t & 1) * S * PITCH;
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                const int rr = lw + 3 * y;
                if (rr < S) {
#pragma unroll
                    for (int x = 0; x < NSEG; ++x) c[rr * PITCH + lane + 64 * x] = pre[y * NSEG + x];
                }
            }
            const int f = tid - 64;
            if (f < S) vst[(t & 1) * S + f] = vin;
        };
        load(0);
        commit(0);
        load(1);
        __syncthreads();
        for (int64_t t = 0; t < nchunks; ++t) {
            commit(t + 1);
            __syncthreads();
            load(t + 2);
        }
        return;
    }

    // ------------------------------------------------------- compute wave
    // Steps run in groups of G; the LDS operands of group g+1 (diagonal
    // factor, input, and the KR coefficients each lane pushes) are read while
    // the dependent chain of group g runs.
    constexpr int G = 8;
    struct Grp {
        T d[G], vd[G], cf[G][KR];
    };
    __syncthreads();
    T acc[KR];
#pragma unroll
    for (int s = 0; s < KR; ++s) acc[s] = T(0);

    for (int64_t t = 0; t < nchunks; ++t) {
        const T *c = cst + (t & 1) * S * PITCH;
        const T *vv = vst + (t & 1) * S;
        for (int g = 0; g < S / 64; ++g) {
            const int64_t jb = t * S + 64 * g;        // first step of this 64-block
            if (jb >= nb) break;
            const int ulim = (int)min((int64_t)64, nb - jb);
            auto load = [&](int u0, Grp &q) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const int u = min(u0 + e, 63);
                    const T *crow = c + (64 * g + u) * PITCH;
                    q.d[e] = DIAG ? crow[0] : T(1);
                    q.vd[e] = vv[64 * g + u] * q.d[e];
#pragma unroll
                    for (int s = 0; s < KR; ++s) {
                        // step offset of slot (s, lane).  Offsets > K read a
                        // zero slot; offsets <= 0 occur only for s = 0 in lanes
                        // whose step is already done, where the value is unused.
                        const int m = 64 * s + lane - u;
                        q.cf[e][s] = crow[min(max(m, 0), PITCH - 1)];
                    }
                }
            };
            T ov = T(0);
            auto run = [&](int u0, const Grp &q) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const int u = u0 + e;
                    if (u < ulim) {
                        const T x = fma(acc[0], q.d[e], q.vd[e]);   // acc = -pending
                        const T xb = lane_bcast(x, u);
#pragma unroll
                        for (int s = 0; s < KR; ++s) acc[s] = fma(-q.cf[e][s], xb, acc[s]);
                        ov = lane == u ? xb : ov;
                    }
                }
            };
            Grp ga, gb;
            load(0, ga);
            for (int u0 = 0; u0 < ulim; u0 += 2 * G) {
                load(u0 + G, gb);
                run(u0, ga);
                load(u0 + 2 * G, ga);
                run(u0 + G, gb);
            }
            const int64_t st = jb + lane;
            if (st < nb) {
                const int64_t r = s0 + row_of(st);
                if (a.dout) a.dout[r] = (double)ov;
                else a.tout[r] = ov;
            }
#pragma unroll
            for (int s = 0; s < KR - 1; ++s) acc[s] = acc[s + 1];
            acc[KR - 1] = T(0);
        }
        __syncthreads();
    }
}

template <typename T, int KR, int S, bool FWD, bool DIAG>
static hipError_t launch_sweep_cfg(const SweepArgs<T> &a, hipStream_t s)
{
    const size_t lds = (2 * (size_t)S * (64 * (KR - 1) + 8) + 2 * S) * sizeof(T);
    auto kern = k_sweep<T, KR, S, FWD, DIAG>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.pt.p), dim3(256), lds, s, a);
    return hipGetLastError();
}

// chunks of 64 steps: two LDS buffers of 64 rows of pitch 64*(KR-1)
template <typename T, int KR>
static hipError_t launch_sweep_kr(const SweepArgs<T> &a, hipStream_t s)
{
    if (a.fwd) {
        if (a.diag) return launch_sweep_cfg<T, KR, 64, true, true>(a, s);
        return launch_sweep_cfg<T, KR, 64, true, false>(a, s);
    }
    if (a.diag) return launch_sweep_cfg<T, KR, 64, false, true>(a, s);
    return launch_sweep_cfg<T, KR, 64, false, false>(a, s);
}

template <>
hipError_t launch_sweep<float>(const SweepArgs<float> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (k < 64) return launch_sweep_kr<float, 2>(a, s);
    if (k < 128) return launch_sweep_kr<float, 3>(a, s);
    if (k < 192) return launch_sweep_kr<float, 4>(a, s);
    return launch_sweep_kr<float, 5>(a, s);
}

template <>
hipError_t launch_sweep<double>(const SweepArgs<double> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (k < 64) return launch_sweep_kr<double, 2>(a, s);
    if (k < 128) return launch_sweep_kr<double, 3>(a, s);
    return hipErrorInvalidValue;               // FP64 factors support K <= 127
}

}  // namespace sap
