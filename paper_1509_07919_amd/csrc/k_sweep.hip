#include <utility>
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
// MI355X design.  One workgroup per block (or per row chunk of a block, see
// below): wave 0 runs the dependent chain, seven loader waves stage the
// coefficient rows and the inputs of the coming chunks of 32 steps in LDS.
// A chunk's rows are one contiguous, 16-byte aligned run in HBM (row pitch
// CP), so it is copied with 16-byte global_load_lds, 1 KiB per instruction,
// into one of up to 8 LDS buffers (as many as fit two workgroups per CU);
// each loader wave owns every seventh chunk, has at most that one in flight
// and waits only for its own copies.  The chain itself needs few bytes per
// step, so what sets the pace is how many chunks are in flight per CU.
// The pending sums acc_{j+1..j+K} live in wave 0's VGPRs: register s, lane l holds the step
// 64*s + l counted from the start of the current 64-step block; KR = 1 +
// ceil(K/64) registers cover the reach of step 63 of the block (63 + K), and
// the registers shift down by one every 64 steps, so register indices stay
// static for any K <= 255.
// Per step: one FMA for x_j (lane u holds the result), a v_readlane
// broadcast (lane index in an SGPR), and one FMA per register in every lane.
// A lane's pending sum is final once its step is reached (later steps push
// zeros to it), so the outputs of a 64-step block are formed at its end and
// written 64 at a time, coalesced.
//
// Chunked form (sap_internal.h): the same chain runs over one row chunk per
// workgroup, so a block's sweep has nch chains in flight instead of one.  The
// zero-state pass ends by reading the K pending sums out of the register ring
// (its outgoing state q(c)).  In the circular kernels below, each workgroup
// of the from-state pass then chains the state entering its own chunk,
// p_in(c+1) = q(c) + X(c) p_in(c), from the first chunk of its block, while
// its first staging copies are in flight: the kernel boundary makes every
// q visible, and no workgroup waits for another.  The ring kernel (K > 56)
// has the last zero-state workgroup of each block (atomic ticket) chain all
// the block's states instead.  The from-state pass seeds the ring with -p_in
// and writes the outputs.
#include "sap_internal.h"
#include "dev_common.h"

namespace sap {

// Waves per sweep workgroup: one compute wave and kSweepWaves - 1 loaders.
constexpr int kSweepWaves = 4;

// Chains the chunk states of block blk over the first nlink links after
// chunk c0 (the first chunk in the sweep direction), NW waves, K < 64: wave
// w sums the terms i in [IW w, IW w + IW) of X(c)^T p for output slot
// m = lane, IW = 64 / NW.  On return sh[0..64) holds the state entering
// chunk c0 + dir (nlink + 1) (zero past K); STORE also writes every state
// to a.st.  A non-null top gives chunk c0 the incoming state -top (K
// entries), which adds the link of chunk c0 itself.
//
// The chain runs in FP64 whatever the factor precision: the transfer
// matrices are FP64 and each link q(c) + X(c)^T p is formed in FP64.  A
// transfer matrix and the terms of a link can be much larger than the state
// they produce (weak dominance makes the homogeneous recurrence grow inside a
// chunk), and FP32 rounding of those terms would then dominate the sweep's
// own FP32 error.
//
// NR > 1: the states of right-hand sides col0 .. col0+nc-1 are chained at
// once (multi-RHS sweeps), each transfer matrix read once for all of them;
// sh[64 j ..] then holds column j's state.  q, st and top are per column
// (strides p*nch*K, p*nch*K and p*K).
template <typename T, bool FWD, int NW, bool STORE, int NR = 1, int H = 1>
__device__ void chain_states(const SweepArgs<T> &a, int blk, int nchb, int nlink, double *sh,
                             const T *top = nullptr, int col0 = 0, int nc = 1)
{
    // H output slots per lane (m = lane + 64 h, K < 64 H); wave w sums the
    // terms i in [IW w, IW w + IW) of X(c)^T p
    constexpr int W64 = 64 * H;
    constexpr int IW = W64 / NW;
    const int k = a.pt.k;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)blk * a.nch;
    const int64_t qs = (int64_t)a.pt.p * a.nch * k;     // column stride of q and st
    const int64_t ts = (int64_t)a.pt.p * k;             // column stride of top
    const T *qc = a.q + col0 * qs;
    double *cur = sh;             // [NR][W64] state entering the current chunk
    double *part = sh + W64 * NR; // [NW][NR][W64] partial sums
    const int c0 = FWD ? 0 : nchb - 1;            // chunk whose q seeds the chain
    const int dir = FWD ? 1 : -1;
    // the state entering chunk c0 + dir is q(c0), or with an incoming state
    // -top the chain starts one link earlier, from -top entering chunk c0
    const int first = top ? c0 : c0 + dir;        // chunk of the first link
    if (top) ++nlink;
    if (tid < 64) {
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int m = 64 * h + tid;
                double v = 0.0;
                if (j < nc && m < k)
                    v = top ? -(double)top[j * ts + m] : (double)qc[j * qs + (base + c0) * k + m];
                cur[j * W64 + m] = v;
                if (STORE && !top && j < nc && m < k)
                    a.st[(col0 + j) * qs + (base + c0 + dir) * k + m] = v;
            }
    }
    // the transfer matrices of NG links are loaded at once, so their
    // latencies overlap; the links are then chained one after the other (with
    // two slots per lane, one link at a time and one slot's half of X at a
    // time, which keeps the registers of the sweep kernels that chain)
    constexpr int NG = H > 1 ? 1 : (NR > 1 ? 2 : ((sizeof(T) == 8 || NW > 4) ? (STORE ? 2 : 3) : 4));
    auto load_x = [&](int c, int h, double (&dst)[IW]) {
        const double *x = a.xf + (base + c) * k * k;
#pragma unroll
        for (int e = 0; e < IW; ++e) {
            const int i = IW * wave + e;
            dst[e] = (i < k && 64 * h + lane < k) ? x[i * k + 64 * h + lane] : 0.0;
        }
    };
    __syncthreads();
    for (int g = 0; g < nlink; g += NG) {
        double xg[NG][IW], qg[NG][NR][H];
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int c = first + dir * (g + j);
            if (g + j < nlink) {
                if (H == 1) load_x(c, 0, xg[j]);
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int h = 0; h < H; ++h)
                        qg[j][r][h] = (wave == 0 && 64 * h + lane < k && r < nc)
                                          ? (double)qc[r * qs + (base + c) * k + 64 * h + lane] : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            if (g + j < nlink) {
                const int c = first + dir * (g + j);         // chunk of this link
#pragma unroll 1
                for (int h = 0; h < H; ++h) {
                    if (H > 1) load_x(c, h, xg[j]);
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const double *cr = cur + r * W64 + IW * wave;
                        double s0 = 0.0, s1 = 0.0;
#pragma unroll
                        for (int e = 0; e < IW; e += 2) {
                            s0 = fma(xg[j][e], cr[e], s0);
                            s1 = fma(xg[j][e + 1], cr[e + 1], s1);
                        }
                        part[(wave * NR + r) * W64 + 64 * h + lane] = s0 + s1;
                    }
                }
                __syncthreads();
                if (wave == 0) {
#pragma unroll
                    for (int r = 0; r < NR; ++r)
#pragma unroll
                        for (int h = 0; h < H; ++h) {
                            const int m = 64 * h + lane;
                            double ps[NW];
#pragma unroll
                            for (int w = 0; w < NW; ++w) ps[w] = part[(w * NR + r) * W64 + m];
#pragma unroll
                            for (int hh = NW / 2; hh >= 1; hh /= 2)
#pragma unroll
                                for (int w = 0; w < hh; ++w) ps[w] += ps[w + hh];
                            const double v = qg[j][r][h] + ps[0];
                            cur[r * W64 + m] = m < k ? v : 0.0;
                            if (STORE && m < k && r < nc)
                                a.st[(col0 + r) * qs + (base + c + dir) * k + m] = v;
                        }
                }
                __syncthreads();
            }
        }
    }
}

// End of a zero-state workgroup: the last of a block's workgroups to arrive
// (atomic ticket) chains the block's chunk states.
template <typename T, bool FWD, int NW, int H = 1>
__device__ void chain_if_last(const SweepArgs<T> &a, int blk, int nchb, double *scratch)
{
    __shared__ int last_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                        // publish this chunk's q
        const unsigned old = atomicAdd(a.ticket + blk, 1u);
        last_sh = old == (unsigned)(a.nch - 1);
    }
    __syncthreads();
    if (!last_sh) return;
    __threadfence();                            // see every chunk's q
    if (nchb >= 2) chain_states<T, FWD, NW, true, 1, H>(a, blk, nchb, nchb - 2, scratch);
    if (threadIdx.x == 0) a.ticket[blk] = 0u;   // ready for the next sweep
}

// Rows of one staged chunk, and the LDS of a sweep workgroup: nbuf staging
// buffers of S coefficient rows (pitch CP, the HBM layout) and nbuf buffers
// of S prescaled inputs v*d.
constexpr int kSweepRows = 32;
template <typename T>
static size_t sweep_lds_bytes(int cp, int nbuf, int h = 1)
{
    const size_t b = ((size_t)nbuf * kSweepRows * cp + (size_t)nbuf * kSweepRows) * sizeof(T);
    // chain_states scratch: h slots of 64 per lane
    const size_t chain = (size_t)64 * h * (kSweepWaves + 1) * sizeof(double);
    return b > chain ? b : chain;
}

template <typename T, int KR, bool FWD, bool DIAG, int PH>
// two workgroups per CU: kSweepWaves / 2 waves per SIMD
__global__ __launch_bounds__(64 * kSweepWaves, kSweepWaves / 2) void k_sweep(SweepArgs<T> a, int nbuf)
{
    constexpr int NL = kSweepWaves - 1;               // loader waves
    constexpr int S = kSweepRows;
    static_assert(S == 32, "a chunk is half a 64-step block");
    static_assert(KR >= 2, "ring must cover 64 + K slots");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = a.pt.k;
    const int CP = coef_pitch(k, (int)sizeof(T));
    T *stage = reinterpret_cast<T *>(smem_raw);       // [nbuf][S][CP]
    T *vst = stage + (size_t)nbuf * S * CP;           // [nbuf][S]

    const int blk = PH == SWEEP_WHOLE ? (int)blockIdx.x : (int)(blockIdx.x % a.pt.p);
    const int ch = PH == SWEEP_WHOLE ? 0 : (int)(blockIdx.x / a.pt.p);
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    // rows [r0, r1) of the block handled here
    const int nchb = PH == SWEEP_WHOLE ? 1 : (int)((nb + a.clen - 1) / a.clen);
    const int64_t r0 = PH == SWEEP_WHOLE ? 0 : min((int64_t)ch * a.clen, nb);
    const int64_t r1 = PH == SWEEP_WHOLE ? nb : min(r0 + a.clen, nb);
    const int64_t nst = r1 - r0;
    // a chunk hands a state on if a chunk follows it in the sweep direction
    const bool passes = ch < nchb && (FWD ? ch + 1 < nchb : ch > 0);
    const bool receives = ch < nchb && (FWD ? ch > 0 : ch + 1 < nchb);
    if (PH == SWEEP_FROM_STATE && ch >= nchb) return;      // empty chunk
    // the zero-state pass has nothing to run for the last chunk of a sweep,
    // but its workgroup still takes part in the block's ticket
    const int nchunks = (PH == SWEEP_ZERO_STATE && !passes) ? 0 : (int)((nst + S - 1) / S);
    // chunks staged ahead of the one being swept (nbuf is 2..NL+1)
    const int depth = nbuf - 1;
    const T *dtop = (a.dtop && blk > 0) ? a.dtop + (int64_t)blk * k : nullptr;
    const T *dbot = (a.dbot && blk < a.pt.p - 1) ? a.dbot + (int64_t)blk * k : nullptr;

    // row of the block handled at step t, and the staged row of step uc of a
    // chunk (a backward chunk is staged in row order, so its steps run from
    // the last staged row up)
    auto row_of = [&](int64_t t) -> int64_t { return FWD ? r0 + t : r1 - 1 - t; };
    auto ridx = [&](int uc) { return FWD ? uc : S - 1 - uc; };
    auto count = [&](int t) { return (int)min((int64_t)S, nst - (int64_t)t * S); };

    if (wave != 0) {
        // ------------------------------------------------------ loaders
        // Loader wave lw owns the chunks t = lw (mod NL).  A chunk is one
        // contiguous, 16-byte aligned run of cnt*CP entries in HBM, copied
        // straight into LDS with 16-byte global_load_lds (1 KiB per
        // instruction), together with its inputs.  The owner waits for its
        // own copies only (it has no others in flight), zeroes the staged rows
        // past the chunk's end (their steps then push nothing), stores v*d,
        // and meets the compute wave at the barrier before that chunk.
        const int lw = __builtin_amdgcn_readfirstlane(wave - 1);
        T vin = T(0);
        auto issue = [&](int t) {
            const int cnt = count(t);
            const int64_t rlo = FWD ? r0 + (int64_t)t * S : r1 - (int64_t)t * S - cnt;
            const unsigned char *src =
                reinterpret_cast<const unsigned char *>(a.F + (s0 + rlo) * CP);
            unsigned char *dst = reinterpret_cast<unsigned char *>(
                stage + ((size_t)(t % nbuf) * S + (FWD ? 0 : S - cnt)) * CP);
            const int nbytes = cnt * CP * (int)sizeof(T);
            for (int q = 0; q * 1024 < nbytes; ++q) {
                const int off = q * 1024 + lane * 16;
                if (off < nbytes)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(src + off),
                        (__attribute__((address_space(3))) void *)(dst + q * 1024), 16, 0, 0);
            }
            vin = T(0);
            if (lane < cnt) {
                const int64_t r = row_of((int64_t)t * S + lane);
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
        };
        auto finish = [&](int t) {
            const int cnt = count(t);
            T *buf = stage + (size_t)(t % nbuf) * S * CP;
            if (cnt < S) {
                T *z = buf + (FWD ? cnt : 0) * CP;
                for (int i = lane; i < (S - cnt) * CP; i += 64) z[i] = T(0);
            }
            if (lane < S) {
                T d = T(1);
                if (DIAG && lane < cnt) d = buf[ridx(lane) * CP];
                vst[(t % nbuf) * S + lane] = lane < cnt ? vin * d : T(0);
            }
        };
        // A zero-state chunk in the middle of a block will have its transfer
        // matrix X read by the block's chaining workgroup: touch its lines
        // now so that read hits the L2 (a block's chunks share blockIdx mod
        // P, hence the XCD when P is a multiple of the XCD count).
        T pf = T(0);
        if (PH == SWEEP_ZERO_STATE && passes && receives) {
            const int64_t xbytes = (int64_t)k * k * (int64_t)sizeof(double);
            const int64_t off = (int64_t)(lw * 64 + lane) * 128;
            if (off < xbytes)
                pf = *reinterpret_cast<const T *>(
                    reinterpret_cast<const unsigned char *>(a.xf + ((int64_t)blk * a.nch + ch) * k * k) + off);
        }
        if (lw < depth && lw < nchunks) issue(lw);
        for (int t = 0; t < nchunks; ++t) {
            if (t % NL == lw) {
                __builtin_amdgcn_s_waitcnt(0);        // this wave's copies of chunk t
                finish(t);
            }
            __syncthreads();                          // chunk t staged; chunk t-1 swept
            const int tn = t + depth;                 // goes to the buffer of chunk t-1
            if (tn < nchunks && tn % NL == lw) issue(tn);
        }
        asm volatile("" ::"v"(pf));                   // keeps the prefetch load
    } else {
        // ------------------------------------------------------- compute wave
        // Steps run in groups of G; the KR coefficients each lane pushes for
        // group g+1 are read from LDS while the dependent chain of group g
        // runs.  Rows past the chunk's end are zero, so groups run whole.
        // Lane l keeps d and v*d of step l of the current 64-step block in
        // registers (loaded with the chunk that holds it), so the step itself
        // is one FMA in lane u.  Offsets m <= 0 (lanes whose step is done, and
        // lane u itself) read the zero slot K+1 like offsets m > K, so a done
        // lane's pending sum stays final and the outputs of the block are
        // formed at its end, again one FMA per lane.
        constexpr int G = 4;
        static_assert(S % (2 * G) == 0, "groups tile the chunk");
        struct Grp {
            T cf[G][KR];
        };
        T acc[KR];
#pragma unroll
        for (int s = 0; s < KR; ++s) {
            // a chunk that receives a state starts from acc = -p_in
            const int m = 64 * s + lane;
            acc[s] = (PH == SWEEP_FROM_STATE && receives && m < k)
                         ? (T)(-a.st[((int64_t)blk * a.nch + ch) * k + m]) : T(0);
        }

        T dl = T(0), vdl = T(0);                      // step `lane` of the 64-block
        for (int t = 0; t < nchunks; ++t) {
            __syncthreads();                          // chunk t staged
            const T *buf = stage + (size_t)(t % nbuf) * S * CP;
            // the staged steps t*S .. t*S+cnt-1 are steps ub .. ub+cnt-1 of the
            // 64-step block that starts at step jb
            const int ub = (t * S) & 63;
            const int64_t jb = (int64_t)t * S - ub;
            const int cnt = count(t);
            const int ulim = ub + cnt;
            if (lane >= ub && lane < ub + S) {
                const int uc = lane - ub;
                dl = DIAG ? buf[ridx(uc) * CP] : T(1);
                vdl = vst[(t % nbuf) * S + uc];
            }
            auto load = [&](int u0, Grp &q) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const int uc = min(u0 + e, S - 1);       // staged step
                    const int u = ub + uc;                    // step in the 64-block
                    // slots 1..K+1 of the row: offset m maps to slot
                    // min(m - 1, K) + 1 taken unsigned, which is K+1 (zero)
                    // for m <= 0 and m > K
                    const T *crow1 = buf + ridx(uc) * CP + 1;
                    const int m1 = lane - 1 - u;
#pragma unroll
                    for (int s = 0; s < KR; ++s)
                        q.cf[e][s] = crow1[min((unsigned)(m1 + 64 * s), (unsigned)k)];
                }
            };
            auto run = [&](int u0, const Grp &q) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    const int u = ub + u0 + e;
                    const T x = fma(acc[0], dl, vdl);        // x_u in lane u (acc = -pending)
                    const T xb = lane_bcast(x, u);
#pragma unroll
                    for (int s = 0; s < KR; ++s) acc[s] = fma(-q.cf[e][s], xb, acc[s]);
                }
            };
            Grp ga, gb;
            load(0, ga);
            for (int u0 = 0; u0 < cnt; u0 += 2 * G) {
                load(u0 + G, gb);
                run(u0, ga);
                load(u0 + 2 * G, ga);
                run(u0 + G, gb);
            }
            const bool last = (int64_t)t * S + cnt == nst;
            if (ulim == 64 || last) {
                const int64_t st = jb + lane;
                if (PH != SWEEP_ZERO_STATE && lane < ulim) {
                    const T ov = fma(acc[0], dl, vdl);     // x of step `lane`
                    const int64_t r = s0 + row_of(st);
                    if (a.dout) a.dout[r] = (double)ov;
                    else a.tout[r] = ov;
                }
                if (PH == SWEEP_ZERO_STATE && last) {
                    // outgoing state: pending sums of the K steps after the
                    // chunk, slots ulim .. ulim+K-1 of the ring before it shifts
#pragma unroll
                    for (int s = 0; s < KR; ++s) {
                        const int m = 64 * s + lane - ulim;
                        if (m >= 0 && m < k) a.q[((int64_t)blk * a.nch + ch) * k + m] = -acc[s];
                    }
                }
#pragma unroll
                for (int s = 0; s < KR - 1; ++s) acc[s] = acc[s + 1];
                acc[KR - 1] = T(0);
            }
        }
    }
    if constexpr (PH == SWEEP_ZERO_STATE && KR <= 3)   // chunked up to K = 127
        chain_if_last<T, FWD, kSweepWaves, KR - 1>(a, blk, nchb, reinterpret_cast<double *>(stage));
}

// ------------------------------------------------ circular form, K <= 56
// The same chain with the pending sums in ONE register per lane: lane l
// holds the step j with j = l (mod 64), a ring of 64 slots that covers the
// K + 1 live sums when K < 64.  Step u pushes x_u to lane l with the
// coefficient of offset m = (l - u) mod 64, which is zero unless 1 <= m <= K.
// Loader waves copy a chunk's compact rows into LDS with 16-byte
// global_load_lds as above, then rotate each row into that lane order: lane
// m reads offset m of the row (offset 0 and offsets past K read the row's
// zero slot K+1) and writes it to lane (u + m) mod 64 of the step's 64-entry
// line, so every line is written whole, zeros included.  The compute wave
// then reads one LDS word per step at a fixed offset, with no index
// arithmetic: per step one FMA for x_u, the v_readlane broadcast and one FMA
// per lane.  A lane's sum is final once its step is reached and receives
// nothing more until step u + 64 - K starts the next use of the slot; so
// every G = 8 steps the lanes of the group's steps take their outputs and
// clear their slots, which needs G <= 64 - K.
constexpr int kCircMaxK = 56;
constexpr int kCircG = 8;
template <typename T>
constexpr int circ_waves() { return sizeof(T) == 8 ? 4 : 8; }   // one compute wave, the rest load
template <typename T>
static size_t circ_lds_bytes(int cp, int nr)
{
    constexpr int NS = circ_waves<T>() - 1;           // one staging buffer per loader
    // [2][S][64] rotated lines, [NR][2][S] v*d, [2][S] d, [NR][NW+1][64] FP64
    // chain scratch and [NS][S][CP] staged rows
    return ((size_t)2 * kSweepRows * 64 + 2 * (size_t)(nr + 1) * kSweepRows +
            (size_t)NS * kSweepRows * cp) * sizeof(T) +
           (size_t)64 * nr * (circ_waves<T>() + 1) * sizeof(double);
}

// NR > 1: right-hand sides c0 .. c0+NR-1 (c0 = NR * blockIdx.y, those below
// a.m) in one workgroup: every staged coefficient row serves all of them and
// the compute wave runs NR independent chains, interleaved step by step.
template <typename T, bool FWD, bool DIAG, int PH, int NR>
__global__ __launch_bounds__(64 * circ_waves<T>(), circ_waves<T>() / 2) void k_sweep_circ(SweepArgs<T> a)
{
    constexpr int S = kSweepRows;
    constexpr int G = kCircG;
    constexpr int NW = circ_waves<T>();
    constexpr int NL = NW - 1;
    static_assert(S % (2 * G) == 0, "groups tile the chunk");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = a.pt.k;
    const int CP = coef_pitch(k, (int)sizeof(T));
    T *gsh = reinterpret_cast<T *>(smem_raw);         // [2][S][64]
    T *vst = gsh + 2 * S * 64;                        // [NR][2][S]
    T *dsh = vst + 2 * S * NR;                        // [2][S]
    double *csh = reinterpret_cast<double *>(dsh + 2 * S);   // [NR][NW+1][64] FP64 chain scratch
    T *stage = reinterpret_cast<T *>(csh + NR * (NW + 1) * 64);   // [NL][S][CP], 16-byte aligned
    const int c0 = NR * (int)blockIdx.y;              // first right-hand side
    const int nc = min(NR, a.m - c0);                 // right-hand sides here
    const int64_t ldv = a.ldv;

    const int blk = PH == SWEEP_WHOLE ? (int)blockIdx.x : (int)(blockIdx.x % a.pt.p);
    const int ch = PH == SWEEP_WHOLE ? 0 : (int)(blockIdx.x / a.pt.p);
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int nchb = PH == SWEEP_WHOLE ? 1 : (int)((nb + a.clen - 1) / a.clen);
    const int64_t r0 = PH == SWEEP_WHOLE ? 0 : min((int64_t)ch * a.clen, nb);
    const int64_t r1 = PH == SWEEP_WHOLE ? nb : min(r0 + a.clen, nb);
    const int64_t nst = r1 - r0;
    const bool passes = ch < nchb && (FWD ? ch + 1 < nchb : ch > 0);
    const bool receives = ch < nchb && (FWD ? ch > 0 : ch + 1 < nchb);
    if (PH == SWEEP_FROM_STATE && ch >= nchb) return;
    const int nchunks = (PH == SWEEP_ZERO_STATE && !passes) ? 0 : (int)((nst + S - 1) / S);
    // boundary deltas of right-hand side c0 + j: dtop/dbot + j * dstr
    const int64_t dstr = (int64_t)a.pt.p * k;
    const T *dtop = (a.dtop && blk > 0) ? a.dtop + (int64_t)c0 * dstr + (int64_t)blk * k : nullptr;
    const T *dbot = (a.dbot && blk < a.pt.p - 1) ? a.dbot + (int64_t)c0 * dstr + (int64_t)blk * k : nullptr;
    auto row_of = [&](int64_t t) -> int64_t { return FWD ? r0 + t : r1 - 1 - t; };
    auto ridx = [&](int uc) { return FWD ? uc : S - 1 - uc; };
    auto count = [&](int t) { return (int)min((int64_t)S, nst - (int64_t)t * S); };
    // The state entering this chunk, chained by the whole workgroup from the
    // outgoing states q of the chunks before it in the sweep direction and
    // their transfer matrices (all written by earlier launches), while the
    // first staging copies are in flight; it lands in csh[64 j ..] for
    // right-hand side c0 + j.
    // dtop as the incoming state -dtop of the block's first chunk (forward)
    const T *top = (FWD && a.top_as_state) ? dtop : nullptr;
    auto entering_state = [&]() {
        chain_states<T, FWD, NW, false, NR>(a, blk, nchb, FWD ? ch - 1 : nchb - 2 - ch, csh, top,
                                            c0, nc);
    };

    if (wave != 0) {
        // ------------------------------------------------------ loaders
        // Loader wave lw owns the chunks t = lw (mod NL) and its staging
        // buffer lw; it has at most one chunk in flight.  After its copies of
        // chunk t land it rotates the rows into the line buffer t mod 2
        // (free: the compute wave finished chunk t-2 before the previous
        // barrier), stores d and v*d and meets the compute wave at the
        // barrier before chunk t; then it refills its staging buffer with
        // chunk t + NL, off that critical path.
        const int lw = __builtin_amdgcn_readfirstlane(wave - 1);
        T *sbuf = stage + (size_t)lw * S * CP;
        T vin[NR];
        auto issue = [&](int t) {
            const int cnt = count(t);
            const int64_t rlo = FWD ? r0 + (int64_t)t * S : r1 - (int64_t)t * S - cnt;
            const unsigned char *src =
                reinterpret_cast<const unsigned char *>(a.F + (s0 + rlo) * CP);
            unsigned char *dst = reinterpret_cast<unsigned char *>(sbuf + (FWD ? 0 : S - cnt) * CP);
            const int nbytes = cnt * CP * (int)sizeof(T);
            for (int q = 0; q * 1024 < nbytes; ++q) {
                const int off = q * 1024 + lane * 16;
                if (off < nbytes)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(src + off),
                        (__attribute__((address_space(3))) void *)(dst + q * 1024), 16, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) vin[j] = T(0);
            if (lane < cnt) {
                const int64_t r = row_of((int64_t)t * S + lane);
                const T *dt = top ? nullptr : dtop;    // top enters as a state
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    if (j >= nc) break;
                    const int64_t o = (int64_t)(c0 + j) * ldv + s0 + r;
                    if (a.xin) {
                        double x = a.xin[o];
                        if (dt && r < k) x += (double)dt[j * dstr + r];
                        if (dbot && r >= nb - k) x += (double)dbot[j * dstr + r - (nb - k)];
                        vin[j] = (T)x;
                    } else {
                        T x = a.tin[o];
                        if (dt && r < k) x += dt[j * dstr + r];
                        if (dbot && r >= nb - k) x += dbot[j * dstr + r - (nb - k)];
                        vin[j] = x;
                    }
                }
            }
        };
        // offset this lane reads from every row: m = lane, or the zero slot
        // K+1 for m = 0 and m > K
        const int mi = (int)min((unsigned)(lane - 1), (unsigned)k) + 1;
        auto finish = [&](int t) {
            const int cnt = count(t);
            const int lu = lane + ((t * S) & 63);
            T *g = gsh + (t & 1) * S * 64;
            // all reads first (rows past the chunk's end hold stale data and
            // are written as zeros), so their latencies overlap
            T v[S];
#pragma unroll
            for (int uc = 0; uc < S; ++uc) v[uc] = sbuf[ridx(uc) * CP + mi];
#pragma unroll
            for (int uc = 0; uc < S; ++uc) g[uc * 64 + ((lu + uc) & 63)] = uc < cnt ? v[uc] : T(0);
            if (lane < S) {
                // steps past the chunk's end get d = 0 and v*d = 0: x = 0
                const T d = lane < cnt ? (DIAG ? sbuf[ridx(lane) * CP] : T(1)) : T(0);
#pragma unroll
                for (int j = 0; j < NR; ++j) vst[(j * 2 + (t & 1)) * S + lane] = vin[j] * d;
                dsh[(t & 1) * S + lane] = d;
            }
        };
        if (lw < nchunks) issue(lw);
        if (PH == SWEEP_FROM_STATE && receives) entering_state();
        for (int t = 0; t < nchunks; ++t) {
            const bool own = t % NL == lw;
            if (own) {
                __builtin_amdgcn_s_waitcnt(0);        // this wave's copies of chunk t
                finish(t);
            }
            __syncthreads();                          // chunk t rotated; chunk t-1 swept
            // the staging buffer was read before the barrier: refill it
            if (own && t + NL < nchunks) issue(t + NL);
        }
    } else {
        // ------------------------------------------------------- compute wave
        if (PH == SWEEP_FROM_STATE && receives) entering_state();
        // acc = -(incoming pending sums): the chained state, or top in the
        // first chunk of a block
        T acc[NR], vdl[NR], xo[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            acc[j] = (PH == SWEEP_FROM_STATE && receives) ? (T)(-csh[j * 64 + lane])
                   : (PH == SWEEP_FROM_STATE && top && lane < k && j < nc) ? top[j * dstr + lane]
                                                                           : T(0);
            vdl[j] = T(0);
            xo[j] = T(0);
        }
        T dl = T(0);
        for (int t = 0; t < nchunks; ++t) {
            __syncthreads();                          // chunk t rotated
            const T *g = gsh + (t & 1) * S * 64 + lane;
            const int ub = (t * S) & 63;
            const int cnt = count(t);
            if (lane >= ub && lane < ub + S) {
                dl = dsh[(t & 1) * S + lane - ub];
#pragma unroll
                for (int j = 0; j < NR; ++j) vdl[j] = vst[(j * 2 + (t & 1)) * S + lane - ub];
            }
            T ca[G], cb[G];
            auto load = [&](int u0, T (&c)[G]) {
#pragma unroll
                for (int e = 0; e < G; ++e) c[e] = g[(u0 + e) * 64];
            };
            auto run = [&](int u0, const T (&c)[G]) {
#pragma unroll
                for (int e = 0; e < G; ++e) {
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        const T x = fma(acc[j], dl, vdl[j]);     // x_u in lane u (acc = -pending)
                        const T xb = lane_bcast(x, ub + u0 + e);
                        acc[j] = fma(-c[e], xb, acc[j]);
                    }
                }
                // the group's lanes take their outputs and free their slots
                const int d = lane - ub - u0;
                if ((unsigned)d < (unsigned)G && u0 + d < cnt) {
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        xo[j] = fma(acc[j], dl, vdl[j]);
                        acc[j] = T(0);
                    }
                }
            };
            load(0, ca);
#pragma unroll
            for (int u0 = 0; u0 < S; u0 += 2 * G) {
                load(u0 + G, cb);
                run(u0, ca);
                if (u0 + 2 * G < S) load(u0 + 2 * G, ca);
                run(u0 + G, cb);
            }
            if (PH != SWEEP_ZERO_STATE && lane >= ub && lane < ub + cnt) {
                const int64_t r = s0 + row_of((int64_t)t * S + lane - ub);
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    if (j >= nc) break;
                    const int64_t o = (int64_t)(c0 + j) * ldv + r;
                    if (a.dout) a.dout[o] = (double)xo[j];
                    else a.tout[o] = xo[j];
                }
            }
        }
        if (PH == SWEEP_ZERO_STATE && nchunks > 0) {
            // outgoing state: the pending sums of the K steps after the chunk,
            // step nst + m in lane (nst + m) mod 64
            const int m = (lane - (int)(nst & 63)) & 63;
            const int64_t qs = (int64_t)a.pt.p * a.nch * k;
            if (m < k)
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (j < nc) a.q[(c0 + j) * qs + ((int64_t)blk * a.nch + ch) * k + m] = -acc[j];
        }
    }
}

template <typename T, bool FWD, bool DIAG, int PH, int NR>
static hipError_t launch_circ_nr(const SweepArgs<T> &a, hipStream_t s)
{
    const unsigned grid = PH == SWEEP_WHOLE ? a.pt.p : a.pt.p * a.nch;
    const size_t lds = circ_lds_bytes<T>(coef_pitch(a.pt.k, (int)sizeof(T)), NR);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_sweep_circ<T, FWD, DIAG, PH, NR>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid, (unsigned)((a.m + NR - 1) / NR)), dim3(64 * circ_waves<T>()),
                       lds, s, a);
    return hipGetLastError();
}

template <typename T, bool FWD, bool DIAG, int PH>
static hipError_t launch_circ_ph(const SweepArgs<T> &a, hipStream_t s)
{
    if (a.m == 1) return launch_circ_nr<T, FWD, DIAG, PH, 1>(a, s);
    return launch_circ_nr<T, FWD, DIAG, PH, kMultiRhs>(a, s);
}

template <typename T, bool FWD, bool DIAG>
static hipError_t launch_circ_cfg(const SweepArgs<T> &a, hipStream_t s)
{
    if (a.phase == SWEEP_ZERO_STATE) return launch_circ_ph<T, FWD, DIAG, SWEEP_ZERO_STATE>(a, s);
    if (a.phase == SWEEP_FROM_STATE) return launch_circ_ph<T, FWD, DIAG, SWEEP_FROM_STATE>(a, s);
    return launch_circ_ph<T, FWD, DIAG, SWEEP_WHOLE>(a, s);
}

template <typename T>
static hipError_t launch_circ(const SweepArgs<T> &a, hipStream_t s)
{
    if (a.fwd) {
        if (a.diag) return launch_circ_cfg<T, true, true>(a, s);
        return launch_circ_cfg<T, true, false>(a, s);
    }
    if (a.diag) return launch_circ_cfg<T, false, true>(a, s);
    return launch_circ_cfg<T, false, false>(a, s);
}

template <typename T, int KR, bool FWD, bool DIAG, int PH>
static hipError_t launch_sweep_ph(const SweepArgs<T> &a, hipStream_t s)
{
    const int cp = coef_pitch(a.pt.k, (int)sizeof(T));
    const unsigned grid = PH == SWEEP_WHOLE ? a.pt.p : a.pt.p * a.nch;
    // deepest staging (2..kSweepWaves buffers: each loader wave has one
    // chunk in flight) that keeps two workgroups per CU when the grid has
    // more than one workgroup per CU
    const size_t cap = grid > 256 ? kMaxLds / 2 : kMaxLds;
    const int h = KR - 1 < 1 ? 1 : KR - 1;
    int nbuf = kSweepWaves;
    while (nbuf > 2 && sweep_lds_bytes<T>(cp, nbuf, h) > cap) --nbuf;
    const size_t lds = sweep_lds_bytes<T>(cp, nbuf, h);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_sweep<T, KR, FWD, DIAG, PH>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kSweepWaves), lds, s, a, nbuf);
    return hipGetLastError();
}

template <typename T, int KR, bool FWD, bool DIAG>
static hipError_t launch_sweep_cfg(const SweepArgs<T> &a, hipStream_t s)
{
    if constexpr (KR <= 3) {                   // chained states up to K = 127
        if (a.phase == SWEEP_ZERO_STATE)
            return launch_sweep_ph<T, KR, FWD, DIAG, SWEEP_ZERO_STATE>(a, s);
        if (a.phase == SWEEP_FROM_STATE)
            return launch_sweep_ph<T, KR, FWD, DIAG, SWEEP_FROM_STATE>(a, s);
    }
    if (a.phase != SWEEP_WHOLE) return hipErrorInvalidValue;
    return launch_sweep_ph<T, KR, FWD, DIAG, SWEEP_WHOLE>(a, s);
}

template <typename T, int KR>
static hipError_t launch_sweep_kr(const SweepArgs<T> &a, hipStream_t s)
{
    if (a.fwd) {
        if (a.diag) return launch_sweep_cfg<T, KR, true, true>(a, s);
        return launch_sweep_cfg<T, KR, true, false>(a, s);
    }
    if (a.diag) return launch_sweep_cfg<T, KR, false, true>(a, s);
    return launch_sweep_cfg<T, KR, false, false>(a, s);
}

template <>
hipError_t launch_sweep<float>(const SweepArgs<float> &a0, hipStream_t s)
{
    SweepArgs<float> a = a0;          // one right-hand side unless stated
    if (a.m < 1) a.m = 1;
    if (a.ldv == 0) a.ldv = a.pt.n;
    const int k = a.pt.k;
    if (k <= kCircMaxK) return launch_circ<float>(a, s);
    if (a.m > 1) return hipErrorInvalidValue;     // multi-RHS sweeps need K <= 56
    if (k < 64) return launch_sweep_kr<float, 2>(a, s);
    if (k < 128) return launch_sweep_kr<float, 3>(a, s);
    if (k < 192) return launch_sweep_kr<float, 4>(a, s);
    return launch_sweep_kr<float, 5>(a, s);
}

template <>
hipError_t launch_sweep<double>(const SweepArgs<double> &a0, hipStream_t s)
{
    SweepArgs<double> a = a0;          // one right-hand side unless stated
    if (a.m < 1) a.m = 1;
    if (a.ldv == 0) a.ldv = a.pt.n;
    const int k = a.pt.k;
    if (k <= kCircMaxK) return launch_circ<double>(a, s);
    if (a.m > 1) return hipErrorInvalidValue;     // multi-RHS sweeps need K <= 56
    if (k < 64) return launch_sweep_kr<double, 2>(a, s);
    if (k < 128) return launch_sweep_kr<double, 3>(a, s);
    if (k < 192) return launch_sweep_kr<double, 4>(a, s);
    return launch_sweep_kr<double, 5>(a, s);
}

// Coefficient M of a row held as lane M mod 16 of register M / 16 in every
// row of sixteen lanes, broadcast to all lanes (DPP row_newbcast).
template <int M, int NR>
__device__ __forceinline__ double row_bcast(const double (&c)[NR])
{
    return __builtin_amdgcn_mov_dpp(c[M >> 4], 0x150 + (M & 15), 0xf, 0xf, true);
}

// acc + (lane N of the row of sixteen lanes of c) * x, the broadcast folded
// into the FMA (DPP row_newbcast on its first operand).  A DPP read of a VGPR
// needs two wait states after a VALU write of it, which the compiler does not
// track through inline assembly: WAIT inserts them, and xfer_step asks for it
// at the first read of each register of c in a step (c is not written within
// a step).
template <int N, bool WAIT>
__device__ __forceinline__ double fma_row_bcast(double acc, double c, double x)
{
    if (WAIT)
        asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "=v"(acc) : "v"(c), "v"(x), "n"(N), "0"(acc));
    else
        asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "=v"(acc) : "v"(c), "v"(x), "n"(N), "0"(acc));
    return acc;
}

// One step of the transfer recurrence on the pending sums p: p[m-1] = p[m] + c_m x
template <int KM, int NR, int... Ms>
__device__ __forceinline__ void xfer_step(double (&p)[KM], const double (&c)[NR], double x,
                                          std::integer_sequence<int, Ms...>)
{
    ((p[Ms] = fma_row_bcast<(Ms + 1) & 15, Ms == 0 || ((Ms + 1) & 15) == 0>(p[Ms + 1], c[(Ms + 1) >> 4], x),
      ((Ms & 3) == 3 ? __builtin_amdgcn_sched_barrier(0) : (void)0)), ...);
}

// ------------------------------------------------------ transfer matrices
// One workgroup of four waves per chunk that hands a state on (blockIdx.y
// selects the coefficient array).  Wave w takes the w-th quarter of the
// chunk's steps: lane i runs those steps with zero inputs from the incoming
// state e_i (pending sum 1 for the i-th step), so its K pending sums at the
// end form row i of the quarter's transfer X_w.  p[m] holds the pending sum
// of the m-th step after the current one: one step is x = -p[0]*d,
// p[m-1] = p[m] + F[j][m]*x.  Coefficient rows are loaded two rows ahead,
// coefficient m into lane m mod 16 of each row of sixteen lanes, and each FMA
// takes its coefficient through a DPP row broadcast.  The chunk's transfer is
// the product X_0 X_1 X_2 X_3 (a state s maps to s X), formed through two LDS
// slots.  All of it is FP64 for either factor precision (FP32 coefficients
// are widened exactly): see chain_states.
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_sweep_xfer(XferArgs<T> a)
{
    static_assert(KM <= 64, "four registers of sixteen coefficients");
    using DT = double;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    DT *Xs = reinterpret_cast<DT *>(smem_raw);   // [2][K][K]
    const int k = a.pt.k;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int kk = k * k;
    const int arr = blockIdx.y;
    const T *F = a.F[arr];
    const bool fwd = a.fwd[arr] != 0, diag = a.diag[arr] != 0;
    const int blk = (int)(blockIdx.x % a.pt.p), ch = (int)(blockIdx.x / a.pt.p);
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int nchb = (int)((nb + a.clen - 1) / a.clen);
    if (!(ch < nchb && (fwd ? ch + 1 < nchb : ch > 0))) return;
    const int64_t r0 = (int64_t)ch * a.clen, r1 = min(r0 + a.clen, nb);
    const int64_t nst = r1 - r0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t t_lo = nst * wave / 4, t_hi = nst * (wave + 1) / 4;

    DT p[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) p[m] = (m == lane) ? 1.0 : 0.0;
    // coefficient m of a row sits in lane m mod 16 of every row of sixteen
    // lanes (register m / 16, widened to FP64 at the end of an iteration) and
    // reaches all lanes through a row broadcast (DPP row_newbcast) folded into
    // the FMA's operand
    constexpr int NR = (KM + 15) / 16;
    constexpr int D = 2;                 // two rows ahead: three waves a SIMD at K = 50
    DT fr[D][NR];
    T fn[D][NR];
    // raw loads with no branch and no use before the end of an iteration, so
    // their wait sits there: the row is clamped into the chunk (rows past the
    // wave's last step are loaded but never used) and slots past K read slot
    // K + 1, which holds zero
    auto load = [&](int64_t t0, T (&dst)[D][NR]) {
#pragma unroll
        for (int e = 0; e < D; ++e) {
            const int64_t t = t0 + e;
            const int64_t row = min(max(fwd ? r0 + t : r1 - 1 - t, r0), r1 - 1);
#pragma unroll
            for (int r = 0; r < NR; ++r)
                dst[e][r] = F[(s0 + row) * CP + min((lane & 15) + 16 * r, k + 1)];
        }
    };
    auto widen = [&]() {
#pragma unroll
        for (int e = 0; e < D; ++e)
#pragma unroll
            for (int r = 0; r < NR; ++r) fr[e][r] = (DT)fn[e][r];
    };
    auto step = [&](const DT (&c)[NR]) {
        const DT d0 = row_bcast<0>(c);            // unconditional: no branch in a step
        const DT d = diag ? d0 : 1.0;
        const DT x = -p[0] * d;
        xfer_step(p, c, x, std::make_integer_sequence<int, KM - 1>{});
        p[KM - 1] = 0.0;
        __builtin_amdgcn_sched_barrier(0);
    };
    // D steps an iteration (the shift of p is register renaming), then the rest
    load(t_lo, fn);
    widen();
    int64_t t0 = t_lo;
    for (; t0 + D <= t_hi; t0 += D) {
        load(t0 + D, fn);
#pragma unroll
        for (int e = 0; e < D; ++e) step(fr[e]);
        widen();
    }
#pragma unroll
    for (int e = 0; e < D - 1; ++e)
        if (t0 + e < t_hi) step(fr[e]);
    // X = ((X_0 X_1) X_2) X_3 through two K x K slots of LDS (A: the running
    // product, B: the next factor), so the kernel needs 2 K^2 elements of
    // LDS and three workgroups fit on a CU beside the tips kernel; each
    // thread forms a 4 x 4 output block (8 LDS reads per 16 FMAs; rows and
    // columns past K are clamped on read and not written)
    DT *A = Xs, *Bm = Xs + kk;
    auto put = [&](int w, DT *dst) {
        if (wave == w && lane < k) {
            DT *xw = dst + lane * k;
#pragma unroll
            for (int m = 0; m < KM; ++m)
                if (m < k) xw[m] = p[m];
        }
    };
    const int nbk = (k + 3) / 4, nblk = nbk * nbk;     // <= 256 for K <= 64
    auto block_mul = [&](int b, DT (&acc)[4][4]) {
        const int i0 = 4 * (b / nbk), m0 = 4 * (b - (b / nbk) * nbk);
        int ir[4], mc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ir[q] = min(i0 + q, k - 1) * k;
            mc[q] = min(m0 + q, k - 1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
        for (int c = 0; c < k; ++c) {
            DT av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[q] = A[ir[q] + c];
                bv[q] = Bm[c * k + mc[q]];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[r][q] = fma(av[r], bv[q], acc[r][q]);
        }
    };
    auto block_store = [&](DT *dst, int b, const DT (&acc)[4][4]) {
        const int i0 = 4 * (b / nbk), m0 = 4 * (b - (b / nbk) * nbk);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (i0 + r < k && m0 + q < k) dst[(i0 + r) * k + m0 + q] = acc[r][q];
    };
    // waves 2 and 3 park X_2 and X_3 in global scratch (their registers are
    // then free: the kernel keeps few enough VGPRs for three workgroups per
    // CU); they are copied back into slot B when their product comes
    DT *scr = a.scratch + (((int64_t)arr * a.pt.p + blk) * a.nch + ch) * 2 * kk;
    put(0, A);
    put(1, Bm);
    put(2, scr);
    put(3, scr + kk);
    DT acc[4][4];
    for (int w = 2; w <= 4; ++w) {
        __threadfence_block();                    // the parked partials, to this workgroup
        __syncthreads();                          // A and B complete
        if (tid < nblk) block_mul(tid, acc);
        __syncthreads();                          // A and B read
        if (w == 4) break;
        if (tid < nblk) block_store(A, tid, acc);
        for (int e = tid; e < kk; e += 256) Bm[e] = scr[(w - 2) * kk + e];
    }
    DT *out = a.xf[arr] + ((int64_t)blk * a.nch + ch) * kk;
    if (tid < nblk) block_store(out, tid, acc);
}

// Transfer matrices for 64 <= K < 128: one workgroup of two waves per chunk
// that hands a state on; wave h runs the basis states i = 64 h + lane over the
// whole chunk, so no partial transfers are multiplied (the product form above
// would need 2 K^2 FP64 entries of LDS).  A lane keeps the pending sums of the
// next 128 steps in registers.  Each wave copies its coming coefficient rows
// (coefficient m in lane m mod 64 of register m / 64, eight rows ahead) into a
// ring of its own in LDS and reads them back at one address for all lanes.
template <typename T>
__global__ __launch_bounds__(128) void k_sweep_xfer_wide(XferArgs<T> a)
{
    constexpr int KM = 128;
    constexpr int D = 8;
    using DT = double;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = a.pt.k;
    const int CP = coef_pitch(k, (int)sizeof(T));   // row pitch in HBM
    const int arr = blockIdx.y;
    const T *F = a.F[arr];
    const bool fwd = a.fwd[arr] != 0, diag = a.diag[arr] != 0;
    const int blk = (int)(blockIdx.x % a.pt.p), ch = (int)(blockIdx.x / a.pt.p);
    const int64_t s0 = a.pt.starts[blk];
    const int64_t nb = a.pt.starts[blk + 1] - s0;
    const int nchb = (int)((nb + a.clen - 1) / a.clen);
    if (!(ch < nchb && (fwd ? ch + 1 < nchb : ch > 0))) return;
    const int64_t r0 = (int64_t)ch * a.clen, r1 = min(r0 + a.clen, nb);
    const int64_t nst = r1 - r0;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int i = 64 * wave + lane;                 // basis state of this lane
    DT *ring = reinterpret_cast<DT *>(smem_raw) + (size_t)wave * 2 * D * KM;   // [2][D][KM]

    DT p[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) p[m] = (m == i) ? 1.0 : 0.0;
    T fr[D][2], fn[D][2];
    auto load = [&](int64_t t0, T (&dst)[D][2]) {
#pragma unroll
        for (int e = 0; e < D; ++e) {
            const int64_t t = t0 + e;
            const int64_t row = fwd ? r0 + t : r1 - 1 - t;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int m = 64 * q + lane;
                dst[e][q] = (t < nst && m <= k) ? F[(s0 + row) * CP + m] : T(0);
            }
        }
    };
    load(0, fr);
    int g = 0;
    for (int64_t t0 = 0; t0 < nst; t0 += D, ++g) {
        DT *buf = ring + (g & 1) * D * KM;
#pragma unroll
        for (int e = 0; e < D; ++e)
#pragma unroll
            for (int q = 0; q < 2; ++q) buf[e * KM + 64 * q + lane] = (DT)fr[e][q];
        load(t0 + D, fn);
#pragma unroll
        for (int e = 0; e < D; ++e) {
            if (t0 + e < nst) {
                const DT *row = buf + e * KM;
                const DT d = diag ? row[0] : 1.0;
                const DT x = -p[0] * d;
#pragma unroll
                for (int m = 1; m < KM; ++m) p[m - 1] = fma(row[m], x, p[m]);
                p[KM - 1] = 0.0;
            }
        }
#pragma unroll
        for (int e = 0; e < D; ++e) {
            fr[e][0] = fn[e][0];
            fr[e][1] = fn[e][1];
        }
    }
    if (i < k) {
        DT *out = a.xf[arr] + ((int64_t)blk * a.nch + ch) * k * k + (int64_t)i * k;
#pragma unroll
        for (int m = 0; m < KM; ++m)
            if (m < k) out[m] = p[m];
    }
}

template <typename T>
static hipError_t launch_xfer_wide(const XferArgs<T> &a, hipStream_t s)
{
    const size_t lds = 2 * 2 * 8 * 128 * sizeof(double);   // each wave's [2][8][128] ring
    auto kern = k_sweep_xfer_wide<T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.pt.p * a.nch, a.narr), dim3(128), lds, s, a);
    return hipGetLastError();
}

template <typename T, int KM>
static hipError_t launch_xfer_km(const XferArgs<T> &a, hipStream_t s)
{
    const size_t lds = 2 * (size_t)a.pt.k * a.pt.k * sizeof(double);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_sweep_xfer<T, KM>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.pt.p * a.nch, a.narr), dim3(256), lds, s, a);
    return hipGetLastError();
}

bool sweep_chunking_supported(int k, bool) { return k >= 1 && k < 128; }
bool sweep_top_state_supported(int k) { return k >= 1 && k <= kCircMaxK; }

template <typename T>
hipError_t launch_sweep_xfer(const XferArgs<T> &a, hipStream_t s)
{
    const int k = a.pt.k;
    if (!sweep_chunking_supported(k, sizeof(T) == 4) || a.nch < 2 || a.narr < 1 || a.narr > 4)
        return hipErrorInvalidValue;
    if (k >= 64) return launch_xfer_wide<T>(a, s);
    // KM >= K + 1 slots: the K pending sums plus the zero that enters
    if (k < 8) return launch_xfer_km<T, 8>(a, s);
    if (k < 16) return launch_xfer_km<T, 16>(a, s);
    if (k < 24) return launch_xfer_km<T, 24>(a, s);
    if (k < 32) return launch_xfer_km<T, 32>(a, s);
    if (k < 40) return launch_xfer_km<T, 40>(a, s);
    if (k < 48) return launch_xfer_km<T, 48>(a, s);
    if (k < 56) return launch_xfer_km<T, 56>(a, s);
    return launch_xfer_km<T, 64>(a, s);
}

template hipError_t launch_sweep_xfer<float>(const XferArgs<float> &, hipStream_t);
template hipError_t launch_sweep_xfer<double>(const XferArgs<double> &, hipStream_t);

}  // namespace sap
