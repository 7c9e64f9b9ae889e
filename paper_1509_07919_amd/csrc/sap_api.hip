// C ABI of libsap: argument validation, workspace layout, the factorization
// sequence and the BiCGStab(2) driver.  The host only sequences kernels and
// reads one device scalar per exit point; all arithmetic runs on the GPU.
#include "sap.h"
#include "sap_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace sap;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                               \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return fail(SAP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t starts, partial, status, ticks, Lc, Uc, Lr, Ur, corner, lwin, B, C, V, W, Rbar, Rlu, Rinv, piv,
        gT, yT, dtop, dbot, kv, dpart, sc, xLc, xUc, xLr, xUr, xscr, sq, sst, ticket, total;
};

bool coupled_active(const sap_options &o) { return o.mode == SAP_COUPLED && o.p > 1 && o.k > 0; }

// right-hand sides a batched solve may take at once (the workspace holds
// that many of every per-right-hand-side vector)
int rhs_cap(const sap_options &o) { return o.nrhs > 1 ? o.nrhs : 1; }

// Workgroups per block of k_block_norm, which covers 64 columns each: the
// grid and the partial-norm array are both sized by this one count.
int norm_chunks(const sap_options &o)
{
    const int64_t maxnb = o.n / o.p + (o.n % o.p ? 1 : 0);
    return (int)((maxnb + 63) / 64);
}

// Chains per block for the triangular sweeps (chunked form, sap_internal.h).
// Automatic choice: about as many sweep workgroups as the chip keeps resident
// (two per CU on 256 CUs: one wave per SIMD each, two waves per SIMD), with
// at least 64 rows per chunk.
struct Chunking {
    int nch, clen;
    bool tails_hold_k;       // every block's last chunk has >= K rows (or is its only chunk)
};
Chunking chunking_for(const sap_options &o)
{
    const int64_t maxnb = o.n / o.p + (o.n % o.p ? 1 : 0);
    const bool fp32 = o.factor_prec == SAP_PREC_FP32;
    Chunking c{1, (int)maxnb, true};
    if (o.sweep_chunks == 1 || !sweep_chunking_supported(o.k, fp32)) return c;
    // automatic: chunked only below K = 64; the transfer matrices of wider
    // bands cost more at factor time (N K^2 FP64 FMA per array, 2 ms at
    // N=200k, K=100) than one solve's sweeps save, so there they are built
    // only when asked for
    if (o.sweep_chunks == 0 && o.k >= 64) return c;
    int64_t want = o.sweep_chunks >= 2 ? o.sweep_chunks : 512 / o.p;
    if (want < 2) return c;
    int64_t clen = (maxnb + want - 1) / want;
    if (clen < 64) clen = 64;
    const int64_t nch = (maxnb + clen - 1) / clen;
    if (nch < 2) return c;
    c.nch = (int)nch;
    c.clen = (int)clen;
    // blocks have maxnb or maxnb - 1 rows (the partition of Sec. 3.1)
    for (int64_t nb = maxnb - 1; nb <= maxnb; ++nb) {
        if (nb < 1) continue;
        const int64_t nchb = (nb + clen - 1) / clen;
        if (nchb > 1 && nb - (nchb - 1) * clen < o.k) c.tails_hold_k = false;
    }
    return c;
}

int validate(const sap_options *o)
{
    if (!o) return fail(SAP_ERR_INVALID, "options pointer is null");
    if (o->n < 1) return fail(SAP_ERR_INVALID, "N must be >= 1");
    if (o->k < 0 || o->k > kMaxK) return fail(SAP_ERR_INVALID, "K must be in [0, 255]");
    if (o->k >= o->n && !(o->n == 1 && o->k == 0))
        return fail(SAP_ERR_INVALID, "K must be < N");
    if (o->p < 1 || (int64_t)o->p > o->n) return fail(SAP_ERR_INVALID, "P must be in [1, N]");
    if (o->mode != SAP_DECOUPLED && o->mode != SAP_COUPLED)
        return fail(SAP_ERR_INVALID, "mode must be SAP_DECOUPLED or SAP_COUPLED");
    if (o->factor_prec != SAP_PREC_FP64 && o->factor_prec != SAP_PREC_FP32)
        return fail(SAP_ERR_INVALID, "factor_prec must be SAP_PREC_FP64 or SAP_PREC_FP32");
    if (o->sweep_chunks < 0) return fail(SAP_ERR_INVALID, "sweep_chunks must be >= 0");
    if (o->nrhs < 0 || o->nrhs > kMaxRhs) return fail(SAP_ERR_INVALID, "nrhs must be in [0, 64]");
    if (o->mode == SAP_COUPLED && o->p > 1 && o->n / o->p < 2 * (int64_t)o->k)
        return fail(SAP_ERR_INVALID, "coupled mode needs floor(N/P) >= 2K");
    if (std::isnan(o->boost_eps)) return fail(SAP_ERR_INVALID, "boost_eps is NaN");
    return SAP_OK;
}

Layout layout_for(const sap_options &o)
{
    Layout L{};
    const int64_t n = o.n;
    const int k = o.k, p = o.p;
    const size_t sf = o.factor_prec == SAP_PREC_FP32 ? 4 : 8;
    const int nchunk = norm_chunks(o);
    const bool cpl = coupled_active(o);
    const size_t kk = (size_t)k * k;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.starts = take(sizeof(int64_t) * (p + 1));
    L.partial = take(sizeof(double) * (size_t)p * nchunk);
    L.status = take(64);
    L.ticks = take(64);          // tips phase clocks (3 x u64)
    const size_t fb = sf * n * coef_pitch(k, (int)sf);   // one factor array
    L.Lc = take(fb);
    L.Uc = take(fb);
    L.Lr = o.adjoint ? take(fb) : 0;
    L.Ur = o.adjoint ? take(fb) : 0;
    const size_t ni = cpl ? (size_t)(p - 1) : 0;
    L.corner = cpl ? take(sf * p * kk) : 0;
    // window slabs of the FP64 wide-band LU, one per LU/UL workgroup
    L.lwin = (sf == 8 && k >= kLuWideMinK) ? take(lu_wide_window_bytes(k) * (cpl ? 2 : 1) * p) : 0;
    L.B = cpl ? take(sf * ni * kk) : 0;
    L.C = cpl ? take(sf * ni * kk) : 0;
    L.V = cpl ? take(sf * ni * kk) : 0;
    L.W = cpl ? take(sf * ni * kk) : 0;
    L.Rbar = cpl ? take(sf * ni * kk) : 0;
    L.Rlu = cpl ? take(sf * ni * kk) : 0;
    L.Rinv = cpl ? take(sf * ni * kk) : 0;
    L.piv = cpl ? take(sizeof(int) * ni * k) : 0;
    const size_t m = rhs_cap(o);
    L.gT = take(sf * n * m);
    L.yT = take(sf * n * m);
    L.dtop = cpl ? take(sf * (size_t)p * k * m) : 0;
    L.dbot = cpl ? take(sf * (size_t)p * k * m) : 0;
    L.kv = take(sizeof(double) * 8 * (size_t)n * m);
    L.dpart = take(sizeof(double) * 3 * kDotBlocks * m);
    L.sc = take(sizeof(double) * kScalars * m);
    const Chunking ck = chunking_for(o);
    if (ck.nch >= 2) {
        const size_t xb = sizeof(double) * (size_t)p * ck.nch * kk;   // FP64 transfer matrices
        L.xLc = take(xb);
        L.xUc = take(xb);
        L.xLr = o.adjoint ? take(xb) : 0;
        L.xUr = o.adjoint ? take(xb) : 0;
        // k_sweep_xfer partials (the kernel for K >= 64 multiplies none)
        L.xscr = k < 64 ? take(2 * xb * (o.adjoint ? 4 : 2)) : 0;
        L.sq = take(2 * sf * (size_t)p * ck.nch * k * m);     // first and second sweep of a D^{-1}
        L.sst = take(sizeof(double) * (size_t)p * ck.nch * k);
        L.ticket = take(sizeof(unsigned) * (size_t)p);
    }
    L.total = off;
    return L;
}

}  // namespace

int sap::api_fail(int code, const std::string &msg) { return fail(code, msg); }

struct sap_handle_ {
    sap_options opt;
    bool coupled, fp32;
    Partition pt;
    int nchunk;
    Chunking ck;             // sweep chains per block
    unsigned char *ws;
    Layout L;
    double *h_slots;         // host view of the result slots
    double *d_slots;         // device address the reduction kernels write them to
    int32_t *h_status;       // host copy of the factorization's status words
    // mapped: h_slots is pinned host memory mapped at d_slots (sap_create);
    // otherwise d_slots is device memory and sync_read copies it into
    // slot_copy (handles without host allocations)
    bool mapped;
    double slot_copy[kHostSlots];
    int32_t status_copy[2];
    const double *a_band;
    bool factored, starts_uploaded;
    hipEvent_t ev[5];        // factor start / after LU / end, solve start / end
    hipEvent_t tev[4];       // around the tips phases (T_BC, T_SPK, T_LUrdcd)
    const CsrDev *csr;       // set during sap_solve_sparse: the Krylov product uses it
    bool phases_valid;       // the last factorization recorded them (profiling on)
    hipStream_t side;        // second stream: transfer matrices beside the tips
    hipEvent_t join;         // the side stream's work joins the main stream
    float t_factor, t_lu, t_tips;
    // per-kernel timing (sap_profile): event pairs recorded around launches
    bool prof;
    std::vector<hipEvent_t> pev;                 // pool, 2 per record
    std::vector<std::pair<int, size_t>> precs;   // (kernel class, pool index)
    double prof_ms[SAP_KERNEL_COUNT];
    int64_t prof_n[SAP_KERNEL_COUNT];

    template <typename T> T *ptr(size_t off) { return reinterpret_cast<T *>(ws + off); }
    // Krylov vector i: an N x nrhs block (column c at + c*N); single solves use column 0
    double *kvec(int i) { return ptr<double>(L.kv) + (size_t)i * opt.n * rhs_cap(opt); }
};

namespace {

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
    sap_handle h;
    int kid;
    hipStream_t s;
    size_t idx = 0;
    bool on = false;
    ProfScope(sap_handle h_, int kid_, hipStream_t s_) : h(h_), kid(kid_), s(s_)
    {
        if (!h->prof) return;
        idx = h->precs.size() * 2;
        while (h->pev.size() < idx + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            h->pev.push_back(e);
        }
        if (hipEventRecord(h->pev[idx], s) != hipSuccess) return;
        on = true;
    }
    ~ProfScope()
    {
        if (!on) return;
        if (hipEventRecord(h->pev[idx + 1], s) == hipSuccess) h->precs.push_back({kid, idx});
    }
};

enum KVec { KV_R0 = 0, KV_R1, KV_R2, KV_U0, KV_U1, KV_U2, KV_RT, KV_T };

// ------------------------------------------------------------------ sweeps
// D^{-1} v (forward then backward sweep).  reuse_q: the previous dinv ran on
// the same input v without dtop/dbot, so its first sweep's zero-state pass
// (q, first half of L.sq, not overwritten since) serves this one, and dtop
// enters the first chunk of each block as its incoming state.
template <typename T>
int dinv(sap_handle h, int trans, const double *xin, const T *dtop, const T *dbot,
         double *dout, T *tout, hipStream_t s, bool reuse_q = false, int m = 1)
{
    if (m > 1 && !sweep_top_state_supported(h->opt.k)) {
        // the ring kernels of wide bands sweep one right-hand side at a time
        // (they never reuse a zero-state pass, so the columns are independent)
        const int64_t n = h->opt.n, pk = (int64_t)h->opt.p * h->opt.k;
        for (int c = 0; c < m; ++c) {
            const int rc = dinv<T>(h, trans, xin + c * n, dtop ? dtop + c * pk : nullptr,
                                   dbot ? dbot + c * pk : nullptr, dout ? dout + c * n : nullptr,
                                   tout ? tout + c * n : nullptr, s, false, 1);
            if (rc) return rc;
        }
        return SAP_OK;
    }
    SweepArgs<T> a1{};
    a1.m = m;
    a1.ldv = h->opt.n;
    a1.pt = h->pt;
    a1.xin = xin;
    a1.dtop = dtop;
    a1.dbot = dbot;
    a1.tout = h->ptr<T>(h->L.yT);
    SweepArgs<T> a2{};
    a2.m = m;
    a2.ldv = h->opt.n;
    a2.pt = h->pt;
    a2.tin = h->ptr<T>(h->L.yT);
    a2.dout = dout;
    a2.tout = tout;
    if (!trans) {            // L (forward, unit) then U (backward)
        a1.F = h->ptr<T>(h->L.Lc); a1.fwd = 1; a1.diag = 0;
        a2.F = h->ptr<T>(h->L.Uc); a2.fwd = 0; a2.diag = 1;
    } else {                 // U^T (forward) then L^T (backward, unit)
        a1.F = h->ptr<T>(h->L.Ur); a1.fwd = 1; a1.diag = 1;
        a2.F = h->ptr<T>(h->L.Lr); a2.fwd = 0; a2.diag = 0;
    }
    if (trans) {
        a1.xf = h->ptr<double>(h->L.xUr);
        a2.xf = h->ptr<double>(h->L.xLr);
    } else {
        a1.xf = h->ptr<double>(h->L.xLc);
        a2.xf = h->ptr<double>(h->L.xUc);
    }
    for (SweepArgs<T> *a : {&a1, &a2}) {
        if (h->ck.nch < 2) {
            a->phase = SWEEP_WHOLE;
            a->nch = 1;
            ProfScope ps(h, SAP_KERNEL_SWEEP, s);
            HIP_TRY(launch_sweep<T>(*a, s));
            continue;
        }
        a->nch = h->ck.nch;
        a->clen = h->ck.clen;
        a->q = h->ptr<T>(h->L.sq) +
               (a == &a1 ? 0 : (size_t)h->opt.p * h->ck.nch * h->opt.k * rhs_cap(h->opt));
        a->st = h->ptr<double>(h->L.sst);
        a->ticket = h->ptr<unsigned>(h->L.ticket);
        // dbot must stay inside each block's last chunk, whose q is not used
        const bool reuse = reuse_q && a == &a1 && sweep_top_state_supported(h->opt.k) &&
                           h->ck.tails_hold_k;
        a->top_as_state = reuse ? 1 : 0;
        if (!reuse) {
            a->phase = SWEEP_ZERO_STATE;
            ProfScope ps(h, SAP_KERNEL_SWEEP, s);
            HIP_TRY(launch_sweep<T>(*a, s));
        }
        a->phase = SWEEP_FROM_STATE;
        {
            ProfScope ps(h, SAP_KERNEL_SWEEP, s);
            HIP_TRY(launch_sweep<T>(*a, s));
        }
    }
    return SAP_OK;
}

template <typename T>
int precond_t(sap_handle h, int trans, const double *r, double *z, hipStream_t s, int m)
{
    if (!h->coupled) return dinv<T>(h, trans, r, nullptr, nullptr, z, nullptr, s, false, m);
    T *g = h->ptr<T>(h->L.gT);
    T *dtop = h->ptr<T>(h->L.dtop), *dbot = h->ptr<T>(h->L.dbot);
    int rc = dinv<T>(h, trans, r, nullptr, nullptr, nullptr, g, s, false, m);
    if (rc) return rc;
    CorrArgs<T> c{};
    c.pt = h->pt;
    c.g = g;
    c.B = h->ptr<T>(h->L.B); c.C = h->ptr<T>(h->L.C);
    c.V = h->ptr<T>(h->L.V); c.W = h->ptr<T>(h->L.W);
    c.Rinv = h->ptr<T>(h->L.Rinv);
    c.dtop = dtop; c.dbot = dbot;
    c.trans = trans;
    c.m = m;
    c.ldg = h->opt.n;
    {
        ProfScope ps(h, SAP_KERNEL_CORR, s);
        HIP_TRY(launch_correction<T>(c, s));
    }
    return dinv<T>(h, trans, r, dtop, dbot, z, nullptr, s, true, m);
}

// z = M^{-1} r for m right-hand sides (N x m blocks, column c at + c*N)
int precond(sap_handle h, int trans, const double *r, double *z, hipStream_t s, int m = 1)
{
    return h->fp32 ? precond_t<float>(h, trans, r, z, s, m)
                   : precond_t<double>(h, trans, r, z, s, m);
}

// y = A v (or b - A v) with the matrix of the solve: the band, or the
// reordered sparse matrix of sap_solve_sparse
hipError_t spmv_op(sap_handle h, const double *v, const double *b, double *y, int trans, int m,
                   hipStream_t s)
{
    if (h->csr) return launch_csr_spmv(*h->csr, v, b, y, s);
    return launch_spmv_multi(h->a_band, h->opt.n, h->opt.k, v, b, y, trans, m, s);
}

// Krylov operator  v -> M^{-1} A v  (or M^{-T} A^T v), m right-hand sides
int apply_op(sap_handle h, int trans, const double *v, double *out, hipStream_t s, int m = 1)
{
    double *t = h->kvec(KV_T);
    {
        ProfScope ps(h, SAP_KERNEL_SPMV, s);
        HIP_TRY(spmv_op(h, v, nullptr, t, trans, m, s));
    }
    return precond(h, trans, t, out, s, m);
}

// columns of the current batched solve (1 and none frozen for single solves)
struct Batch {
    int m = 1;
    uint64_t frozen = 0;
};

DotArgs dot_args(sap_handle h, int op, const Batch &bt = Batch())
{
    DotArgs d{};
    d.m = bt.m;
    d.ld = h->opt.n;
    d.frozen = bt.frozen;
    d.n = h->opt.n;
    d.partial = h->ptr<double>(h->L.dpart);
    d.sc = h->ptr<double>(h->L.sc);
    d.host = h->d_slots;
    d.op = op;
    return d;
}

int dots(sap_handle h, int op, std::initializer_list<std::pair<const double *, const double *>> pr,
         hipStream_t s, const int *status = nullptr, const Batch &bt = Batch())
{
    DotArgs d = dot_args(h, op, bt);
    d.status = status;
    int i = 0;
    for (auto &p : pr) { d.x[i] = p.first; d.y[i] = p.second; ++i; }
    d.nd = i;
    ProfScope ps(h, SAP_KERNEL_KRYLOV, s);
    HIP_TRY(launch_dots(d, s));
    return SAP_OK;
}

int update(sap_handle h, int kind, double *x, int op, int nd, hipStream_t s,
           const Batch &bt = Batch())
{
    UpdArgs u{};
    u.kind = kind;
    u.n = h->opt.n;
    u.x = x;
    u.r0 = h->kvec(KV_R0); u.r1 = h->kvec(KV_R1); u.r2 = h->kvec(KV_R2);
    u.u0 = h->kvec(KV_U0); u.u1 = h->kvec(KV_U1); u.u2 = h->kvec(KV_U2);
    u.rt = h->kvec(KV_RT);
    u.dots = dot_args(h, op, bt);
    u.dots.nd = nd;
    ProfScope ps(h, SAP_KERNEL_KRYLOV, s);
    HIP_TRY(launch_update(u, s));
    return SAP_OK;
}

int sync_read(sap_handle h, hipStream_t s, double *nrm2, double *brk)
{
    if (!h->mapped)
        HIP_TRY(hipMemcpyAsync(h->h_slots, h->d_slots, sizeof(double) * kHostSlots * rhs_cap(h->opt),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *nrm2 = h->h_slots[H_NRM2];
    *brk = h->h_slots[H_BREAK];
    return SAP_OK;
}

int read_factor_status(sap_handle h, hipStream_t s, int32_t *nboost, int32_t *singular)
{
    HIP_TRY(hipMemcpyAsync(h->h_status, h->ptr<int>(h->L.status), 2 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *nboost = h->h_status[0];
    *singular = h->h_status[1];
    return SAP_OK;
}

#define TRY(expr)                 \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ < 0) return rc_;  \
    } while (0)

// Factorization times from its events; called once the solve has synchronized
// (the factorization finished before it), so it adds no host round trip.
static void collect_factor_times(sap_handle h)
{
    if (h->t_factor >= 0.0f || !h->ev[2]) return;
    if (hipEventSynchronize(h->ev[2]) != hipSuccess) return;
    (void)hipEventElapsedTime(&h->t_factor, h->ev[0], h->ev[2]);
    (void)hipEventElapsedTime(&h->t_lu, h->ev[0], h->ev[1]);
    (void)hipEventElapsedTime(&h->t_tips, h->ev[1], h->ev[2]);
}

// Left-preconditioned BiCGStab(2), x0 = 0.
int krylov(sap_handle h, int trans, const double *b, double *x, double tol, int32_t maxit,
           hipStream_t s, sap_stats *st)
{
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!b || !x) return fail(SAP_ERR_INVALID, "null vector pointer");
    if (!(tol > 0.0)) return fail(SAP_ERR_INVALID, "tol must be > 0");
    if (maxit < 1) return fail(SAP_ERR_INVALID, "maxit must be >= 1");
    if (trans && !h->opt.adjoint)
        return fail(SAP_ERR_STATE, "handle was created without adjoint = 1");
    const int64_t n = h->opt.n;
    if ((const void *)b < (const void *)(x + n) && (const void *)x < (const void *)(b + n))
        return fail(SAP_ERR_INVALID, "b and x overlap");

    sap_stats loc{};
    if (h->ev[3]) HIP_TRY(hipEventRecord(h->ev[3], s));
    double *r0 = h->kvec(KV_R0), *r1 = h->kvec(KV_R1), *r2 = h->kvec(KV_R2);
    double *u0 = h->kvec(KV_U0), *u1 = h->kvec(KV_U1), *u2 = h->kvec(KV_U2);
    double *rt = h->kvec(KV_RT), *t = h->kvec(KV_T);
    const double *A = h->a_band;
    const int k = h->opt.k;
    double nrm2 = 0, brk = 0;

    // The factorization's status and ||b|| go to host slots now and are read
    // at the first exit test, with its round trip: a singular factorization
    // or b = 0 then ends the solve there (the first quarter step has run on
    // them, and x is reset for b = 0).
    TRY(dots(h, OP_BNORM, {{b, b}}, s, h->ptr<int>(h->L.status)));
    double bnorm = -1.0;           // read at the first exit test
    HIP_TRY(launch_fill(x, 0.0, n, s));
    auto finish = [&](int code, const char *msg) {
        if (h->ev[4]) {
            HIP_TRY(hipEventRecord(h->ev[4], s));
            HIP_TRY(hipEventSynchronize(h->ev[4]));
            HIP_TRY(hipEventElapsedTime(&loc.t_solve_ms, h->ev[3], h->ev[4]));
        } else {
            HIP_TRY(hipStreamSynchronize(s));
        }
        collect_factor_times(h);
        loc.t_factor_ms = h->t_factor;
        loc.t_lu_ms = h->t_lu;
        loc.t_tips_ms = h->t_tips;
        loc.iters = loc.n_apply / 4.0;
        if (st) *st = loc;
        if (code != SAP_OK && code != SAP_NOT_CONVERGED) return fail(code, msg);
        if (code == SAP_NOT_CONVERGED) g_err = msg;
        return code;
    };
    // r0 = M^{-1} b, rt = r0, u0 = 0, scalars reset; the norm of r0 is read
    // at the first exit test (host slot H_NRM0), saving a round trip
    TRY(precond(h, trans, b, r0, s));
    TRY(update(h, UPD_RESTART, x, OP_INIT, 2, s));
    double pnorm0 = 0.0, thr = 0.0, pstart = 0.0;
    bool started = false;          // H_NRM0 of the last (re)start read
    bool first_start = true;       // no restart yet
    bool tn_pending = false;       // H_TRUE of the last restart not read yet
    double tn_restart = 0.0;       // true residual norm at the last restart
    int napply = 0;
    // Reliable updates (Sleijpen and van der Vorst 1996): with FP32 factors
    // the recursive residual stops tracking the true one near FP32 accuracy,
    // so once it has dropped by this factor since the last (re)start the true
    // residual is tested and the iteration restarted from it.
    const double reliable = h->fp32 ? 1e-4 : 0.0;

    // recursive residuals at the last two exit tests since the (re)start
    double pn_last = 0.0, pn_last2 = 0.0;
    int pn_hist = 0;
    // exit test: returns 1 = converged, 2 = restarted, 0 = continue, < 0 error
    // (described by `why`)
    const char *why = "breakdown in BiCGStab(2)";
    auto exit_test = [&]() -> int {
        // When this test may converge or restart (the first after a
        // (re)start, or when the last two tests extrapolate below the
        // threshold), t = b - A x and its norm are enqueued before the
        // synchronization: a converged test then needs no second round trip,
        // and a restart reuses t.  Otherwise they are left out.
        bool spec = !started;
        if (started && pn_hist >= 2 && pn_last2 > 0.0) {
            const double est = pn_last * (pn_last / pn_last2);
            spec = est <= thr || est <= reliable * pstart;
        }
        if (spec) {
            {
                ProfScope ps(h, SAP_KERNEL_SPMV, s);
                HIP_TRY(spmv_op(h, x, b, t, trans, 1, s));            // t = b - A x
            }
            TRY(dots(h, OP_SPEC, {{t, t}}, s));
        }
        TRY(sync_read(h, s, &nrm2, &brk));
        if (bnorm < 0.0) {
            loc.n_boosted = (int32_t)h->h_slots[H_NBOOST];
            if (const int32_t singular = (int32_t)h->h_slots[H_SING]) {
                napply = 0;
                why = singular == 1 ? "zero pivot in a diagonal block (boosting disabled)"
                                    : "singular reduced matrix Rbar";
                return SAP_ERR_SINGULAR;
            }
            bnorm = std::sqrt(h->h_slots[H_BNORM]);
            if (bnorm == 0.0) {                                  // x = 0, no step counted
                HIP_TRY(launch_fill(x, 0.0, n, s));
                napply = 0;
                return 1;
            }
        }
        if (tn_pending) {
            tn_restart = std::sqrt(h->h_slots[H_TRUE]);
            loc.rel_resid_true = tn_restart / bnorm;
            tn_pending = false;
        }
        if (!started) {
            pstart = std::sqrt(h->h_slots[H_NRM0]);
            if (first_start) {
                pnorm0 = pstart;
                thr = tol * pnorm0;
                first_start = false;
            } else {
                thr = tol * bnorm * pstart / tn_restart;
            }
            started = true;
            pn_hist = 0;
        }
        if (brk != 0.0) return SAP_ERR_BREAKDOWN;
        if (!std::isfinite(nrm2)) return SAP_ERR_BREAKDOWN;
        const double pn = std::sqrt(nrm2);
        loc.rel_resid_precond = pn / pnorm0;
        pn_last2 = pn_last;
        pn_last = pn;
        ++pn_hist;
        if (pn > thr && !(pn <= reliable * pstart)) return 0;
        if (spec) {
            // t and its norm are already here: test, else restart from t
            const double tn = std::sqrt(h->h_slots[H_SPEC]);
            loc.rel_resid_true = tn / bnorm;
            if (loc.rel_resid_true <= tol) return 1;
            TRY(precond(h, trans, t, r0, s));
            ++napply;
            ++loc.restarts;
            TRY(update(h, UPD_RESTART, x, OP_INIT, 2, s));
            started = false;
            tn_restart = tn;
            return 2;
        }
        {
            ProfScope ps(h, SAP_KERNEL_SPMV, s);
            HIP_TRY(spmv_op(h, x, b, t, trans, 1, s));            // t = b - A x
        }
        if (pn > thr) {
            // reliable update before the recursive residual reached the
            // tolerance: restart from the true residual without testing it on
            // the host; its norm is read at the next exit test
            TRY(dots(h, OP_TRUE, {{t, t}}, s));
            TRY(precond(h, trans, t, r0, s));
            ++napply;
            ++loc.restarts;
            TRY(update(h, UPD_RESTART, x, OP_INIT, 2, s));
            started = false;
            tn_pending = true;
            return 2;
        }
        TRY(dots(h, OP_NORM, {{t, t}}, s));
        double tn2 = 0, b2 = 0;
        TRY(sync_read(h, s, &tn2, &b2));
        const double tn = std::sqrt(tn2);
        loc.rel_resid_true = tn / bnorm;
        if (loc.rel_resid_true <= tol) return 1;
        TRY(precond(h, trans, t, r0, s));                        // restart
        ++napply;
        ++loc.restarts;
        TRY(update(h, UPD_RESTART, x, OP_INIT, 2, s));
        started = false;                                         // read at the next test
        tn_restart = tn;
        return 2;
    };

    int code = SAP_NOT_CONVERGED;
    for (int32_t it = 0; it < maxit; ++it) {
        int e;
        // j = 0
        TRY(update(h, UPD_U0, x, 0, 0, s));
        TRY(apply_op(h, trans, u0, u1, s)); ++napply;
        TRY(dots(h, OP_GAMMA, {{u1, rt}}, s));
        TRY(update(h, UPD_J0, x, OP_EXIT, 1, s));
        loc.n_apply = napply;
        e = exit_test(); loc.n_apply = napply;
        if (e < 0) return finish(e, why);
        if (e == 1) { code = SAP_OK; break; }
        if (e == 2) continue;
        TRY(apply_op(h, trans, r0, r1, s)); ++napply;
        // j = 1
        TRY(dots(h, OP_RHO, {{r1, rt}}, s));
        TRY(update(h, UPD_U01, x, 0, 0, s));
        TRY(apply_op(h, trans, u1, u2, s)); ++napply;
        TRY(dots(h, OP_GAMMA, {{u2, rt}}, s));
        TRY(update(h, UPD_J1, x, OP_EXIT, 1, s));
        loc.n_apply = napply;
        e = exit_test(); loc.n_apply = napply;
        if (e < 0) return finish(e, why);
        if (e == 1) { code = SAP_OK; break; }
        if (e == 2) continue;
        TRY(apply_op(h, trans, r1, r2, s)); ++napply;
        // minimal-residual part
        TRY(dots(h, OP_MR1, {{r1, r1}, {r0, r1}, {r2, r1}}, s));
        TRY(update(h, UPD_MR2, x, OP_MR2, 2, s));
        TRY(update(h, UPD_FINAL, x, OP_FINAL, 2, s));
        loc.n_apply = napply;
        e = exit_test(); loc.n_apply = napply;
        if (e < 0) return finish(e, why);
        if (e == 1) { code = SAP_OK; break; }
    }
    loc.n_apply = napply;
    if (code == SAP_OK) {
        loc.converged = 1;
        return finish(SAP_OK, "");
    }
    {
        ProfScope ps(h, SAP_KERNEL_SPMV, s);
        HIP_TRY(spmv_op(h, x, b, t, trans, 1, s));
    }
    TRY(dots(h, OP_NORM, {{t, t}}, s));
    double tn2 = 0;
    TRY(sync_read(h, s, &tn2, &brk));
    loc.rel_resid_true = std::sqrt(tn2) / bnorm;
    return finish(SAP_NOT_CONVERGED, "maximum number of iterations reached");
}

// BiCGStab(2) on m right-hand sides at once (columns of B and X, N apart),
// x0 = 0.  Every operator application, dot product and vector update runs
// once for all columns (the SpMV and the sweeps read A and the factors once
// per kMultiRhs columns); each column keeps its own recurrence scalars.  The
// columns run in lockstep: a converged column is frozen (its x is final and
// its updates are skipped), and when a candidate exit of any column fails its
// true-residual test, every active column restarts from its own true
// residual, so that all stay at the same step of the cycle.  A column's
// iteration count is the number of operator applications made while it was
// active, over 4.
int krylov_batch(sap_handle h, const double *B, double *X, int m, double tol, int32_t maxit,
                 hipStream_t s, sap_stats *st)
{
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!B || !X) return fail(SAP_ERR_INVALID, "null matrix pointer");
    if (m < 1 || m > rhs_cap(h->opt))
        return fail(SAP_ERR_INVALID, "m must be in [1, nrhs of the handle]");
    if (!(tol > 0.0)) return fail(SAP_ERR_INVALID, "tol must be > 0");
    if (maxit < 1) return fail(SAP_ERR_INVALID, "maxit must be >= 1");
    const int64_t n = h->opt.n;
    const int64_t tot = n * m;
    if ((const void *)B < (const void *)(X + tot) && (const void *)X < (const void *)(B + tot))
        return fail(SAP_ERR_INVALID, "B and X overlap");
    std::vector<sap_stats> loc(m);
    if (h->ev[3]) HIP_TRY(hipEventRecord(h->ev[3], s));
    double *r0 = h->kvec(KV_R0), *r1 = h->kvec(KV_R1), *r2 = h->kvec(KV_R2);
    double *u0 = h->kvec(KV_U0), *u1 = h->kvec(KV_U1), *u2 = h->kvec(KV_U2);
    double *rt = h->kvec(KV_RT), *t = h->kvec(KV_T);
    const double *A = h->a_band;
    const int k = h->opt.k;
    Batch bt;
    bt.m = m;
    auto slot = [&](int c, int i) { return h->h_slots[(size_t)c * kHostSlots + i]; };
    double nrm2 = 0, brk = 0;
    TRY(dots(h, OP_NORM, {{B, B}}, s, h->ptr<int>(h->L.status), bt));
    TRY(sync_read(h, s, &nrm2, &brk));
    for (int c = 0; c < m; ++c) loc[c].n_boosted = (int32_t)slot(0, H_NBOOST);
    if (const int32_t singular = (int32_t)slot(0, H_SING)) {
        if (st) std::copy(loc.begin(), loc.end(), st);
        return fail(SAP_ERR_SINGULAR, singular == 1 ? "zero pivot in a diagonal block (boosting disabled)"
                                                    : "singular reduced matrix Rbar");
    }
    std::vector<double> bnorm(m), pnorm0(m), thr(m), pstart(m), tnr(m);
    std::vector<int> napply(m, 0), started(m, 0), first(m, 1);
    for (int c = 0; c < m; ++c) {
        bnorm[c] = std::sqrt(slot(c, H_NRM2));
        if (bnorm[c] == 0.0) {                 // x = 0 solves it
            loc[c].converged = 1;
            bt.frozen |= 1ull << c;
        }
    }
    HIP_TRY(launch_fill(X, 0.0, tot, s));
    const double reliable = h->fp32 ? 1e-4 : 0.0;
    int code = SAP_NOT_CONVERGED;
    const char *msg = "maximum number of iterations reached";
    auto all_frozen = [&]() { return bt.frozen == (m == 64 ? ~0ull : ((1ull << m) - 1)); };
    auto count_apply = [&]() {
        for (int c = 0; c < m; ++c)
            if (!((bt.frozen >> c) & 1)) ++napply[c];
    };
    auto finish = [&](int rc, const char *why) {
        if (h->ev[4]) {
            HIP_TRY(hipEventRecord(h->ev[4], s));
            HIP_TRY(hipEventSynchronize(h->ev[4]));
        } else {
            HIP_TRY(hipStreamSynchronize(s));
        }
        float ms = 0.0f;
        if (h->ev[4]) HIP_TRY(hipEventElapsedTime(&ms, h->ev[3], h->ev[4]));
        collect_factor_times(h);
        for (int c = 0; c < m; ++c) {
            loc[c].t_solve_ms = ms;
            loc[c].t_factor_ms = h->t_factor;
            loc[c].t_lu_ms = h->t_lu;
            loc[c].t_tips_ms = h->t_tips;
            loc[c].n_apply = napply[c];
            loc[c].iters = napply[c] / 4.0;
        }
        if (st) std::copy(loc.begin(), loc.end(), st);
        if (rc != SAP_OK && rc != SAP_NOT_CONVERGED) return fail(rc, why);
        if (rc == SAP_NOT_CONVERGED) g_err = why;
        return rc;
    };
    if (all_frozen()) return finish(SAP_OK, "");
    // restart every active column from R (the initial start: R = B)
    auto restart = [&](const double *R) -> int {
        TRY(precond(h, 0, R, r0, s, m));
        count_apply();
        TRY(update(h, UPD_RESTART, X, OP_INIT, 2, s, bt));
        for (int c = 0; c < m; ++c) started[c] = 0;
        return SAP_OK;
    };
    TRY(restart(B));
    for (int c = 0; c < m; ++c) napply[c] = 0;            // the first M^{-1} b is not counted
    // exit test of all active columns: 1 all converged, 2 restarted, 0 go on
    auto exit_test = [&]() -> int {
        TRY(sync_read(h, s, &nrm2, &brk));
        bool any_cand = false;
        std::vector<int> cand(m, 0);
        for (int c = 0; c < m; ++c) {
            if ((bt.frozen >> c) & 1) continue;
            if (!started[c]) {
                pstart[c] = std::sqrt(slot(c, H_NRM0));
                if (first[c]) {
                    pnorm0[c] = pstart[c];
                    thr[c] = tol * pnorm0[c];
                    first[c] = 0;
                } else {
                    thr[c] = tol * bnorm[c] * pstart[c] / tnr[c];
                }
                started[c] = 1;
            }
            const double bk = slot(c, H_BREAK), pn2 = slot(c, H_NRM2);
            if (bk != 0.0 || !std::isfinite(pn2)) return SAP_ERR_BREAKDOWN;
            const double pn = std::sqrt(pn2);
            loc[c].rel_resid_precond = pn / pnorm0[c];
            if (pn <= thr[c] || (reliable > 0.0 && pn <= reliable * pstart[c])) {
                cand[c] = 1;
                any_cand = true;
            }
        }
        if (!any_cand) return 0;
        {
            ProfScope ps(h, SAP_KERNEL_SPMV, s);                  // T = B - A X
            HIP_TRY(launch_spmv_multi(A, n, k, X, B, t, 0, m, s));
        }
        TRY(dots(h, OP_NORM, {{t, t}}, s, nullptr, bt));
        TRY(sync_read(h, s, &nrm2, &brk));
        bool restart_needed = false;
        for (int c = 0; c < m; ++c) {
            if ((bt.frozen >> c) & 1) continue;
            tnr[c] = std::sqrt(slot(c, H_NRM2));
            loc[c].rel_resid_true = tnr[c] / bnorm[c];
            if (cand[c] && loc[c].rel_resid_true <= tol) {
                loc[c].converged = 1;
                bt.frozen |= 1ull << c;
            } else if (cand[c]) {
                restart_needed = true;
            }
        }
        if (all_frozen()) return 1;
        if (!restart_needed) return 0;
        for (int c = 0; c < m; ++c)
            if (!((bt.frozen >> c) & 1)) ++loc[c].restarts;
        TRY(restart(t));
        return 2;
    };
    for (int32_t it = 0; it < maxit; ++it) {
        int e;
        TRY(update(h, UPD_U0, X, 0, 0, s, bt));
        TRY(apply_op(h, 0, u0, u1, s, m)); count_apply();
        TRY(dots(h, OP_GAMMA, {{u1, rt}}, s, nullptr, bt));
        TRY(update(h, UPD_J0, X, OP_EXIT, 1, s, bt));
        e = exit_test();
        if (e < 0) { code = e; msg = "breakdown in BiCGStab(2)"; break; }
        if (e == 1) { code = SAP_OK; break; }
        if (e == 2) continue;
        TRY(apply_op(h, 0, r0, r1, s, m)); count_apply();
        TRY(dots(h, OP_RHO, {{r1, rt}}, s, nullptr, bt));
        TRY(update(h, UPD_U01, X, 0, 0, s, bt));
        TRY(apply_op(h, 0, u1, u2, s, m)); count_apply();
        TRY(dots(h, OP_GAMMA, {{u2, rt}}, s, nullptr, bt));
        TRY(update(h, UPD_J1, X, OP_EXIT, 1, s, bt));
        e = exit_test();
        if (e < 0) { code = e; msg = "breakdown in BiCGStab(2)"; break; }
        if (e == 1) { code = SAP_OK; break; }
        if (e == 2) continue;
        TRY(apply_op(h, 0, r1, r2, s, m)); count_apply();
        TRY(dots(h, OP_MR1, {{r1, r1}, {r0, r1}, {r2, r1}}, s, nullptr, bt));
        TRY(update(h, UPD_MR2, X, OP_MR2, 2, s, bt));
        TRY(update(h, UPD_FINAL, X, OP_FINAL, 2, s, bt));
        e = exit_test();
        if (e < 0) { code = e; msg = "breakdown in BiCGStab(2)"; break; }
        if (e == 1) { code = SAP_OK; break; }
    }
    if (code == SAP_NOT_CONVERGED) {
        // true residuals of the columns still active
        {
            ProfScope ps(h, SAP_KERNEL_SPMV, s);
            HIP_TRY(launch_spmv_multi(A, n, k, X, B, t, 0, m, s));
        }
        TRY(dots(h, OP_NORM, {{t, t}}, s, nullptr, bt));
        TRY(sync_read(h, s, &nrm2, &brk));
        for (int c = 0; c < m; ++c)
            if (!((bt.frozen >> c) & 1)) loc[c].rel_resid_true = std::sqrt(slot(c, H_NRM2)) / bnorm[c];
    }
    return finish(code, code == SAP_OK ? "" : msg);
}

// Preconditioned conjugate gradient (Saad, Alg. 9.1), x0 = 0: the outer loop
// for symmetric positive definite A.  r = b - A x is updated recursively in
// FP64 and z = M^{-1} r uses the handle's preconditioner; one host round
// trip per step reads ||r||^2.  When ||r|| <= tol ||b|| the true residual is
// tested; if it fails, CG restarts from it.
int krylov_cg(sap_handle h, const double *b, double *x, double tol, int32_t maxit, hipStream_t s,
              sap_stats *st)
{
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!b || !x) return fail(SAP_ERR_INVALID, "null vector pointer");
    if (!(tol > 0.0)) return fail(SAP_ERR_INVALID, "tol must be > 0");
    if (maxit < 1) return fail(SAP_ERR_INVALID, "maxit must be >= 1");
    const int64_t n = h->opt.n;
    if ((const void *)b < (const void *)(x + n) && (const void *)x < (const void *)(b + n))
        return fail(SAP_ERR_INVALID, "b and x overlap");
    sap_stats loc{};
    if (h->ev[3]) HIP_TRY(hipEventRecord(h->ev[3], s));
    double *r = h->kvec(KV_R0), *z = h->kvec(KV_R1), *pv = h->kvec(KV_U0), *q = h->kvec(KV_U1);
    double *t = h->kvec(KV_T);
    const double *A = h->a_band;
    const int k = h->opt.k;
    double nrm2 = 0, brk = 0;
    // the factorization's status and ||b|| are read with the first step's
    // round trip (a singular factorization or b = 0 ends the solve there)
    TRY(dots(h, OP_BNORM, {{b, b}}, s, h->ptr<int>(h->L.status)));
    double bnorm = -1.0;
    HIP_TRY(launch_fill(x, 0.0, n, s));
    int napply = 0, steps = 0;
    auto finish = [&](int code, const char *msg) {
        if (h->ev[4]) {
            HIP_TRY(hipEventRecord(h->ev[4], s));
            HIP_TRY(hipEventSynchronize(h->ev[4]));
            HIP_TRY(hipEventElapsedTime(&loc.t_solve_ms, h->ev[3], h->ev[4]));
        } else {
            HIP_TRY(hipStreamSynchronize(s));
        }
        collect_factor_times(h);
        loc.t_factor_ms = h->t_factor;
        loc.t_lu_ms = h->t_lu;
        loc.t_tips_ms = h->t_tips;
        loc.iters = steps;
        loc.n_apply = napply;
        if (st) *st = loc;
        if (code != SAP_OK && code != SAP_NOT_CONVERGED) return fail(code, msg);
        if (code == SAP_NOT_CONVERGED) g_err = msg;
        return code;
    };
    // r = b, z = M^{-1} r, p = z, rho = (r, z)
    HIP_TRY(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    TRY(precond(h, 0, r, z, s));
    ++napply;
    TRY(update(h, UPD_CG_INIT, x, OP_CG_INIT, 2, s));
    int code = SAP_NOT_CONVERGED;
    for (int32_t it = 0; it < maxit; ++it) {
        {
            ProfScope ps(h, SAP_KERNEL_SPMV, s);
            HIP_TRY(spmv_op(h, pv, nullptr, q, 0, 1, s));             // q = A p
        }
        TRY(dots(h, OP_CG_ALPHA, {{pv, q}}, s));
        TRY(update(h, UPD_CG_XR, x, OP_EXIT, 1, s));
        ++steps;
        TRY(sync_read(h, s, &nrm2, &brk));
        if (bnorm < 0.0) {
            loc.n_boosted = (int32_t)h->h_slots[H_NBOOST];
            if (const int32_t singular = (int32_t)h->h_slots[H_SING]) {
                napply = steps = 0;
                return finish(SAP_ERR_SINGULAR, singular == 1
                                                    ? "zero pivot in a diagonal block (boosting disabled)"
                                                    : "singular reduced matrix Rbar");
            }
            bnorm = std::sqrt(h->h_slots[H_BNORM]);
            if (bnorm == 0.0) {                                  // x = 0, no step counted
                HIP_TRY(launch_fill(x, 0.0, n, s));
                napply = steps = 0;
                code = SAP_OK;
                break;
            }
        }
        if (brk != 0.0 || !std::isfinite(nrm2))
            return finish(SAP_ERR_BREAKDOWN, "breakdown in CG (A or M not positive definite)");
        loc.rel_resid_precond = std::sqrt(nrm2) / bnorm;
        if (std::sqrt(nrm2) <= tol * bnorm) {
            {
                ProfScope ps(h, SAP_KERNEL_SPMV, s);
                HIP_TRY(spmv_op(h, x, b, t, 0, 1, s));                     // t = b - A x
            }
            TRY(dots(h, OP_NORM, {{t, t}}, s));
            double tn2 = 0, b2 = 0;
            TRY(sync_read(h, s, &tn2, &b2));
            loc.rel_resid_true = std::sqrt(tn2) / bnorm;
            if (loc.rel_resid_true <= tol) {
                code = SAP_OK;
                break;
            }
            HIP_TRY(hipMemcpyAsync(r, t, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            TRY(precond(h, 0, r, z, s));
            ++napply;
            ++loc.restarts;
            TRY(update(h, UPD_CG_INIT, x, OP_CG_INIT, 2, s));
            continue;
        }
        TRY(precond(h, 0, r, z, s));
        ++napply;
        TRY(dots(h, OP_CG_BETA, {{r, z}}, s));
        TRY(update(h, UPD_CG_P, x, 0, 0, s));
    }
    if (code == SAP_OK) {
        loc.converged = 1;
        return finish(SAP_OK, "");
    }
    {
        ProfScope ps(h, SAP_KERNEL_SPMV, s);
        HIP_TRY(spmv_op(h, x, b, t, 0, 1, s));
    }
    TRY(dots(h, OP_NORM, {{t, t}}, s));
    double tn2 = 0;
    TRY(sync_read(h, s, &tn2, &brk));
    loc.rel_resid_true = std::sqrt(tn2) / bnorm;
    return finish(SAP_NOT_CONVERGED, "maximum number of iterations reached");
}

template <typename T>
int factor_t(sap_handle h, const double *a_band, hipStream_t s)
{
    LuArgs<T> lu{};
    lu.band = a_band;
    lu.pt = h->pt;
    lu.partial = h->ptr<double>(h->L.partial);
    lu.nchunk = h->nchunk;
    double eps = h->opt.boost_eps;
    if (eps == 0.0) eps = h->fp32 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -52);
    lu.boost_eps = eps;
    lu.Lc = h->ptr<T>(h->L.Lc);
    lu.Uc = h->ptr<T>(h->L.Uc);
    lu.Lr = h->opt.adjoint ? h->ptr<T>(h->L.Lr) : nullptr;
    lu.Ur = h->opt.adjoint ? h->ptr<T>(h->L.Ur) : nullptr;
    lu.corner = h->coupled ? h->ptr<T>(h->L.corner) : nullptr;
    lu.status = h->ptr<int>(h->L.status);
    lu.with_ul = h->coupled ? 1 : 0;
    lu.wide = h->L.lwin ? h->ptr<double>(h->L.lwin) : nullptr;
    if (h->coupled && h->prof && h->tev[0])     // tips phase clocks, zeroed ahead of the LU
        HIP_TRY(launch_zero(h->ptr<unsigned long long>(h->L.ticks), 3 * sizeof(unsigned long long), s));
    {
        ProfScope ps(h, SAP_KERNEL_LU, s);
        HIP_TRY(launch_banded_lu<T>(lu, s));
    }
    // the transfer matrices of the chunked sweeps (sap_internal.h) depend only
    // on the factors: they run on the side stream beside the tips
    const bool side = h->ck.nch >= 2 && h->coupled && h->side;
    hipStream_t xs = side ? h->side : s;
    // ev[1] (the LU's end, for its time) also forks the side stream
    if (h->ev[1]) HIP_TRY(hipEventRecord(h->ev[1], s));
    if (side) HIP_TRY(hipStreamWaitEvent(h->side, h->ev[1], 0));
    if (h->ck.nch >= 2) {
        if (!sweep_top_state_supported(h->opt.k))      // ring kernel: per-block tickets
            HIP_TRY(launch_zero(h->ptr<unsigned>(h->L.ticket), sizeof(unsigned) * h->opt.p, xs));
        struct Arr { T *F; size_t xf; int fwd, diag; };
        const Arr arrs[4] = {{lu.Lc, h->L.xLc, 1, 0}, {lu.Uc, h->L.xUc, 0, 1},
                             {lu.Ur, h->L.xUr, 1, 1}, {lu.Lr, h->L.xLr, 0, 0}};
        XferArgs<T> xa{};
        xa.pt = h->pt;
        xa.scratch = h->ptr<double>(h->L.xscr);
        xa.nch = h->ck.nch;
        xa.clen = h->ck.clen;
        for (const Arr &r : arrs) {
            if (!r.F) continue;
            xa.F[xa.narr] = r.F;
            xa.xf[xa.narr] = h->ptr<double>(r.xf);
            xa.fwd[xa.narr] = r.fwd;
            xa.diag[xa.narr] = r.diag;
            ++xa.narr;
        }
        ProfScope ps(h, SAP_KERNEL_XFER, xs);
        HIP_TRY(launch_sweep_xfer<T>(xa, xs));
    }
    if (h->coupled) {
        TipsArgs<T> ta{};
        ta.band = a_band;
        ta.pt = h->pt;
        ta.Lc = lu.Lc; ta.Uc = lu.Uc; ta.corner = lu.corner;
        ta.B = h->ptr<T>(h->L.B); ta.C = h->ptr<T>(h->L.C);
        ta.V = h->ptr<T>(h->L.V); ta.W = h->ptr<T>(h->L.W);
        ta.Rbar = h->ptr<T>(h->L.Rbar); ta.Rlu = h->ptr<T>(h->L.Rlu);
        ta.Rinv = h->ptr<T>(h->L.Rinv);
        ta.piv = h->ptr<int>(h->L.piv);
        ta.status = lu.status;
        // phase clocks and events only while profiling (sap_tips_phase_times)
        const bool phases = h->prof && h->tev[0];
        ta.ticks = phases ? h->ptr<unsigned long long>(h->L.ticks) : nullptr;
        h->phases_valid = phases;
        ProfScope ps(h, SAP_KERNEL_TIPS, s);
        HIP_TRY(launch_tips<T>(ta, s, phases ? h->tev : nullptr));
    }
    if (side) {
        HIP_TRY(hipEventRecord(h->join, h->side));
        HIP_TRY(hipStreamWaitEvent(s, h->join, 0));
    }
    return SAP_OK;
}

// Host state of a handle over a carved workspace.  Allocates nothing; the
// host result slots, events and side stream are added by sap_create.
void init_handle(sap_handle h, const sap_options &o, unsigned char *ws, const Layout &L)
{
    h->opt = o;
    h->coupled = coupled_active(o);
    h->fp32 = o.factor_prec == SAP_PREC_FP32;
    h->ws = ws;
    h->L = L;
    h->pt.n = o.n;
    h->pt.k = o.k;
    h->pt.p = o.p;
    h->pt.maxnb = o.n / o.p + (o.n % o.p ? 1 : 0);
    h->pt.starts = h->ptr<int64_t>(L.starts);
    h->nchunk = norm_chunks(o);
    h->ck = chunking_for(o);
}

int factor_impl(sap_handle h, const double *a_band, hipStream_t s)
{
    if (!h->starts_uploaded) {
        // the partition of Sec. 3.1, and the zero slots after each factor
        // row, which no kernel writes afterwards (fill kernels, not memset
        // nodes, so that the sequence can be captured into a graph)
        HIP_TRY(launch_partition_starts(h->ptr<int64_t>(h->L.starts), h->opt.n, h->opt.p, s));
        const size_t fb = (h->fp32 ? 4 : 8) * (size_t)h->opt.n *
                          coef_pitch(h->opt.k, h->fp32 ? 4 : 8);
        for (size_t off : {h->L.Lc, h->L.Uc, h->L.Lr, h->L.Ur})
            if (off) HIP_TRY(launch_zero(h->ws + off, fb, s));
        h->starts_uploaded = true;
    }
    if (h->ev[0]) HIP_TRY(hipEventRecord(h->ev[0], s));
    {
        ProfScope ps(h, SAP_KERNEL_NORM, s);       // also zeroes the status words
        HIP_TRY(launch_block_norm(a_band, h->pt, h->ptr<double>(h->L.partial), h->nchunk,
                                  h->ptr<int>(h->L.status), s));
    }
    int rc = h->fp32 ? factor_t<float>(h, a_band, s) : factor_t<double>(h, a_band, s);
    if (rc) return rc;
    if (h->ev[2]) HIP_TRY(hipEventRecord(h->ev[2], s));
    h->a_band = a_band;
    h->factored = true;
    h->t_factor = h->t_lu = h->t_tips = -1.0f;
    return SAP_OK;
}

}  // namespace

// Workspace of sap_solve_noalloc: one static array in every GPU's memory
// (each device holds its own copy, at its own address, until the process
// ends).  Host code never passes `scratch` itself to a kernel or a copy: its
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SAP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kSlotBytes = 256;   // result slots ahead of the carved workspace
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices];

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
int scratch_address(unsigned char **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAP_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SAP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        g_scratch[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch[dev];
    return SAP_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *sap_last_error(void) { return g_err.c_str(); }

int sap_workspace_bytes(const sap_options *opt, size_t *bytes)
{
    int rc = validate(opt);
    if (rc) return rc;
    if (!bytes) return fail(SAP_ERR_INVALID, "bytes pointer is null");
    *bytes = layout_for(*opt).total;
    return SAP_OK;
}

int sap_create(const sap_options *opt, void *workspace, size_t ws_bytes, sap_handle *out)
{
    int rc = validate(opt);
    if (rc) return rc;
    if (!out) return fail(SAP_ERR_INVALID, "output handle pointer is null");
    *out = nullptr;
    if (!workspace) return fail(SAP_ERR_INVALID, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(SAP_ERR_INVALID, "workspace must be 256-byte aligned");
    Layout L = layout_for(*opt);
    if (ws_bytes < L.total)
        return fail(SAP_ERR_NOSPACE, "workspace too small: need " + std::to_string(L.total) +
                                         " bytes, got " + std::to_string(ws_bytes));
    sap_handle h = new (std::nothrow) sap_handle_();
    if (!h) return fail(SAP_ERR_INVALID, "out of host memory");
    init_handle(h, *opt, static_cast<unsigned char *>(workspace), L);
    auto cleanup = [&](int code, const std::string &m) {
        if (h->h_slots) (void)hipHostFree(h->h_slots);
        if (h->h_status) (void)hipHostFree(h->h_status);
        for (auto &e : h->ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : h->tev)
            if (e) (void)hipEventDestroy(e);
        if (h->join) (void)hipEventDestroy(h->join);
        if (h->side) (void)hipStreamDestroy(h->side);
        delete h;
        return fail(code, m);
    };
    if (hipHostMalloc((void **)&h->h_slots, sizeof(double) * kHostSlots * rhs_cap(*opt),
                      hipHostMallocMapped) != hipSuccess ||
        hipHostMalloc((void **)&h->h_status, 64, hipHostMallocDefault) != hipSuccess)
        return cleanup(SAP_ERR_HIP, "hipHostMalloc failed");
    if (hipHostGetDevicePointer((void **)&h->d_slots, h->h_slots, 0) != hipSuccess)
        return cleanup(SAP_ERR_HIP, "hipHostGetDevicePointer failed");
    h->mapped = true;
    for (auto &e : h->ev)
        if (hipEventCreate(&e) != hipSuccess) return cleanup(SAP_ERR_HIP, "hipEventCreate failed");
    for (auto &e : h->tev)
        if (hipEventCreate(&e) != hipSuccess) return cleanup(SAP_ERR_HIP, "hipEventCreate failed");
    if (hipEventCreateWithFlags(&h->join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess)
        return cleanup(SAP_ERR_HIP, "creating the side stream failed");
    *out = h;
    return SAP_OK;
}

int sap_factor(sap_handle h, const double *a_band, void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!a_band) return fail(SAP_ERR_INVALID, "a_band is null");
    return factor_impl(h, a_band, static_cast<hipStream_t>(stream));
}

int sap_solve(sap_handle h, const double *b, double *x, double tol, int32_t maxit, void *stream,
              sap_stats *st)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    return krylov(h, 0, b, x, tol, maxit, static_cast<hipStream_t>(stream), st);
}

int sap_solve_adjoint(sap_handle h, const double *g, double *lambda, double tol, int32_t maxit,
                      void *stream, sap_stats *st)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    return krylov(h, 1, g, lambda, tol, maxit, static_cast<hipStream_t>(stream), st);
}

int sap_solve_sparse(sap_handle h, sap_sparse sp, const double *b, double *x, double tol,
                     int32_t maxit, void *stream, sap_stats *st)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    CsrDev m{};
    double *bhat = nullptr, *yhat = nullptr;
    const int32_t *new_row = nullptr, *new_col = nullptr;
    const double *rs = nullptr, *cs = nullptr;
    if (!sparse_plan_parts(sp, &m, &bhat, &yhat, &new_row, &new_col, &rs, &cs))
        return fail(SAP_ERR_STATE, "null plan, or sap_sparse_assemble has not been called");
    if (m.n != h->opt.n || sparse_plan_k(sp) != h->opt.k)
        return fail(SAP_ERR_INVALID, "the handle's N and K must be the plan's");
    if (!b || !x) return fail(SAP_ERR_INVALID, "null vector pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_map_vec(b, new_row, rs, bhat, m.n, 0, s));      // b_hat = P D_r Q b
    h->csr = &m;
    const int rc = krylov(h, 0, bhat, yhat, tol, maxit, s, st);
    h->csr = nullptr;
    if (rc < 0) return rc;
    HIP_TRY(launch_map_vec(yhat, new_col, cs, x, m.n, 1, s));      // x = D_c P^T y_hat
    return rc;
}

int sap_solve_batch(sap_handle h, const double *B, double *X, int32_t m, double tol,
                    int32_t maxit, void *stream, sap_stats *st)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    return krylov_batch(h, B, X, m, tol, maxit, static_cast<hipStream_t>(stream), st);
}

int sap_solve_cg(sap_handle h, const double *b, double *x, double tol, int32_t maxit,
                 void *stream, sap_stats *st)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    return krylov_cg(h, b, x, tol, maxit, static_cast<hipStream_t>(stream), st);
}

int sap_band_grad(sap_handle h, const double *lambda, const double *x, double *g_band,
                  void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!lambda || !x || !g_band) return fail(SAP_ERR_INVALID, "null vector pointer");
    HIP_TRY(launch_band_grad(h->opt.n, h->opt.k, lambda, x, g_band,
                             static_cast<hipStream_t>(stream)));
    return SAP_OK;
}

int sap_solve_noalloc(const sap_options *opt, const double *a_band, const double *b, double *x,
                      double tol, int32_t maxit, void *stream, sap_stats *st)
{
    int rc = validate(opt);
    if (rc) return rc;
    if (opt->adjoint) return fail(SAP_ERR_INVALID, "sap_solve_noalloc needs adjoint = 0");
    if (opt->nrhs > 1) return fail(SAP_ERR_INVALID, "sap_solve_noalloc needs nrhs <= 1");
    if (!a_band || !b || !x) return fail(SAP_ERR_INVALID, "null pointer");
    const Layout L = layout_for(*opt);
    if (L.total > SAP_NOALLOC_SCRATCH_BYTES - kSlotBytes)
        return fail(SAP_ERR_NOSPACE, "sap_solve_noalloc: these options need " +
                                         std::to_string(L.total + kSlotBytes) +
                                         " bytes of scratch; the static scratch holds " +
                                         std::to_string((size_t)SAP_NOALLOC_SCRATCH_BYTES));
    unsigned char *scr = nullptr;
    TRY(scratch_address(&scr));
    // a handle on the stack over the static scratch: no host or device
    // allocation, no events (the statistics carry no device times) and no
    // side stream (the transfer matrices run on `stream`)
    sap_handle_ hs{};
    init_handle(&hs, *opt, scr + kSlotBytes, L);
    hs.d_slots = reinterpret_cast<double *>(scr);
    hs.h_slots = hs.slot_copy;
    hs.h_status = hs.status_copy;
    hs.mapped = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = factor_impl(&hs, a_band, s);
    if (rc) return rc;
    return krylov(&hs, 0, b, x, tol, maxit, s, st);
}

int sap_handle_status(sap_handle h, void *stream, int32_t *n_boosted)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    int32_t nb = 0, sing = 0;
    TRY(read_factor_status(h, static_cast<hipStream_t>(stream), &nb, &sing));
    if (n_boosted) *n_boosted = nb;
    if (sing) return fail(SAP_ERR_SINGULAR, sing == 1 ? "zero pivot in a diagonal block"
                                                      : "singular reduced matrix Rbar");
    return SAP_OK;
}

int sap_spmv(sap_handle h, const double *v, double *y, int32_t trans, void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!v || !y) return fail(SAP_ERR_INVALID, "null vector pointer");
    HIP_TRY(launch_spmv(h->a_band, h->opt.n, h->opt.k, v, nullptr, y, trans ? 1 : 0,
                        static_cast<hipStream_t>(stream)));
    return SAP_OK;
}

int sap_precond_apply(sap_handle h, const double *r, double *z, int32_t trans, void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!r || !z) return fail(SAP_ERR_INVALID, "null vector pointer");
    if (trans && !h->opt.adjoint)
        return fail(SAP_ERR_STATE, "handle was created without adjoint = 1");
    return precond(h, trans ? 1 : 0, r, z, static_cast<hipStream_t>(stream));
}

int sap_get_tips(sap_handle h, int32_t i, double *v, double *w, double *rbar, void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (!h->coupled) return fail(SAP_ERR_STATE, "no interface matrices in this mode");
    if (i < 0 || i >= h->opt.p - 1) return fail(SAP_ERR_INVALID, "interface index out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t kk = (size_t)h->opt.k * h->opt.k;
    const size_t sf = h->fp32 ? 4 : 8;
    std::vector<unsigned char> tmp(kk * sf);
    const size_t offs[3] = {h->L.V, h->L.W, h->L.Rbar};
    double *dst[3] = {v, w, rbar};
    for (int m = 0; m < 3; ++m) {
        if (!dst[m]) continue;
        HIP_TRY(hipMemcpyAsync(tmp.data(), h->ws + offs[m] + (size_t)i * kk * sf, kk * sf,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t e = 0; e < kk; ++e)
            dst[m][e] = h->fp32 ? (double)reinterpret_cast<float *>(tmp.data())[e]
                                : reinterpret_cast<double *>(tmp.data())[e];
    }
    return SAP_OK;
}

int sap_get_factor_rows(sap_handle h, int32_t which, int64_t j0, int64_t count, double *out,
                        void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    if (which < 0 || which > 3) return fail(SAP_ERR_INVALID, "which must be 0..3");
    const size_t offs[4] = {h->L.Lc, h->L.Uc, h->L.Lr, h->L.Ur};
    if (which >= 2 && !h->opt.adjoint)
        return fail(SAP_ERR_STATE, "handle was created without adjoint = 1");
    if (j0 < 0 || count < 0 || j0 + count > h->opt.n || (count > 0 && !out))
        return fail(SAP_ERR_INVALID, "row range out of bounds");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t sf = h->fp32 ? 4 : 8;
    const int k = h->opt.k;
    const int cp = coef_pitch(k, (int)sf);
    std::vector<unsigned char> tmp((size_t)count * cp * sf);
    if (count > 0) {
        HIP_TRY(hipMemcpyAsync(tmp.data(), h->ws + offs[which] + (size_t)j0 * cp * sf, tmp.size(),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    for (int64_t r = 0; r < count; ++r)
        for (int m = 0; m <= k; ++m) {
            const size_t e = (size_t)r * cp + m;
            out[r * (k + 1) + m] = h->fp32 ? (double)reinterpret_cast<float *>(tmp.data())[e]
                                           : reinterpret_cast<double *>(tmp.data())[e];
        }
    return SAP_OK;
}

int sap_tips_phase_times(sap_handle h, double *ms, void *stream)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (!ms) return fail(SAP_ERR_INVALID, "ms is null");
    if (!h->factored) return fail(SAP_ERR_STATE, "sap_factor has not been called");
    ms[0] = ms[1] = ms[2] = 0.0;
    if (!h->coupled) return SAP_OK;
    if (!h->phases_valid)
        return fail(SAP_ERR_STATE, "phase times are recorded only while sap_profile is on");
    HIP_TRY(hipEventSynchronize(h->tev[3]));
    float span = 0.0f;
    HIP_TRY(hipEventElapsedTime(&span, h->tev[0], h->tev[3]));
    if (!tips_in_lds(h->opt.k, h->fp32)) {          // one launch group per phase
        float t1 = 0.0f, t2 = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t1, h->tev[0], h->tev[1]));
        HIP_TRY(hipEventElapsedTime(&t2, h->tev[1], h->tev[2]));
        ms[0] = t1;
        ms[1] = t2;
        ms[2] = span - t1 - t2;
        return SAP_OK;
    }
    // one kernel: its time split by the workgroups' summed phase clocks
    unsigned long long tk[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(tk, h->ptr<unsigned long long>(h->L.ticks), sizeof(tk),
                           hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    const double tot = (double)tk[0] + (double)tk[1] + (double)tk[2];
    for (int q = 0; q < 3; ++q) ms[q] = tot > 0.0 ? span * (double)tk[q] / tot : 0.0;
    return SAP_OK;
}

int sap_profile(sap_handle h, int32_t enable)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (enable) {
        h->precs.clear();
        for (int i = 0; i < SAP_KERNEL_COUNT; ++i) {
            h->prof_ms[i] = 0.0;
            h->prof_n[i] = 0;
        }
    }
    h->prof = enable != 0;
    return SAP_OK;
}

int sap_kernel_time(sap_handle h, int32_t kernel, double *ms, int64_t *launches)
{
    if (!h) return fail(SAP_ERR_INVALID, "null handle");
    if (kernel < 0 || kernel >= SAP_KERNEL_COUNT) return fail(SAP_ERR_INVALID, "bad kernel id");
    if (!h->precs.empty()) {
        HIP_TRY(hipEventSynchronize(h->pev[h->precs.back().second + 1]));
        for (auto &r : h->precs) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, h->pev[r.second], h->pev[r.second + 1]));
            h->prof_ms[r.first] += t;
            h->prof_n[r.first] += 1;
        }
        h->precs.clear();
    }
    if (ms) *ms = h->prof_ms[kernel];
    if (launches) *launches = h->prof_n[kernel];
    return SAP_OK;
}

int sap_destroy(sap_handle h)
{
    if (!h) return SAP_OK;
    for (auto &e : h->pev) (void)hipEventDestroy(e);
    if (h->mapped) {
        (void)hipHostFree(h->h_slots);
        (void)hipHostFree(h->h_status);
    }
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : h->tev)
        if (e) (void)hipEventDestroy(e);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->join) (void)hipEventDestroy(h->join);
    delete h;
    return SAP_OK;
}

}  // extern "C"
