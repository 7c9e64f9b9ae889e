// Sparse front end: the reorderings and the assembly that turn a sparse A
// into the dense banded matrix the SaP preconditioner is built on, and the
// sparse product the outer Krylov loop then uses (arXiv:1509.07919,
// Sec. 3.1 "Diagonal Boosting", "Bandwidth reduction"; Sec. 3.3 the DB and
// CM implementation details; Sec. 3.4 T_DB, T_CM, T_Drop, T_Asmbl).
//
// As in the paper's hybrid design, the combinatorial stages run on the host
// (the paper does DB stages 2-3 and CM stage 3 on the CPU) and the
// data-parallel ones on the GPU:
//   host:  DB  -- minimum-cost perfect bipartite matching with costs
//                 c_ij = log a_i - log |a_ij| (eq:DBrelated), by shortest
//                 augmenting paths (Dijkstra on reduced costs with row and
//                 column potentials) after a greedy match of tight edges;
//                 the potentials give the scaling to an I-matrix;
//          CM  -- Cuthill-McKee on the structure of B + B^T: breadth-first,
//                 neighbours in ascending (degree, index), several starts
//                 (each from the least node of the previous search's last
//                 level), the ordering of least half-bandwidth kept;
//          Drop -- the least K whose outside-the-band entries carry at most
//                 a given fraction of sum |a_ij|;
//          the structure of the reordered matrix (entry map and scales).
//   GPU:   the reordered, scaled values, the dense band (T_Asmbl), the
//          sparse product y = A v inside the Krylov loop, and the maps of
//          the right-hand side and the solution.
// The reordered system:  A_hat = P D_r Q A D_c P^T,  b_hat = P D_r Q b,
// x = D_c P^T y_hat, with Q the DB row permutation and P the CM ordering.
#include "sap.h"
#include "sap_internal.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <limits>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

namespace sap {

// ------------------------------------------------------------ GPU kernels
__global__ void k_sparse_values(const double *__restrict__ vals, const int64_t *__restrict__ src,
                                const double *__restrict__ escale, double *__restrict__ out,
                                int64_t nnz)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256)
        out[e] = vals[src[e]] * escale[e];
}

// band[(K + r - c) N + c] = a_hat[r][c] for |r - c| <= K (entries farther
// out are dropped); the band is zeroed before
__global__ void k_band_from_csr(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                const double *__restrict__ v, int64_t n, int k, double *__restrict__ band)
{
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256)
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            const int64_t c = colidx[e];
            const int64_t d = r - c;
            if (d <= k && d >= -k) band[(k + d) * n + c] = v[e];
        }
}

// y = A v, or y = b - A v: L consecutive lanes per row stride through its
// entries together (loads of neighbouring lanes are neighbouring entries),
// then their partial sums are added across the L lanes
template <int L>
__global__ __launch_bounds__(256) void k_csr_spmv(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const double *__restrict__ a, int64_t n,
                                                  const double *__restrict__ v,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ y)
{
    const int sub = (int)threadIdx.x & (L - 1);
    const int64_t step = (int64_t)gridDim.x * (256 / L);
    for (int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / L; r < n; r += step) {
        double s = 0.0;
        for (int64_t e = rowptr[r] + sub; e < rowptr[r + 1]; e += L) s = fma(a[e], v[colidx[e]], s);
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
        if (sub == 0) y[r] = b ? b[r] - s : s;
    }
}

// out[map[i]] = scale[i] * in[i] (the right-hand side), or
// out[i] = scale[i] * in[map[i]] (the solution)
__global__ void k_map_vec(const double *__restrict__ in, const int32_t *__restrict__ map,
                          const double *__restrict__ scale, double *__restrict__ out, int64_t n,
                          int gather)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (gather) out[i] = scale[i] * in[map[i]];
        else out[map[i]] = scale[i] * in[i];
    }
}

static unsigned grid_for(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 4096);
}

template <int L>
static hipError_t launch_csr_spmv_l(const CsrDev &m, const double *v, const double *b, double *y,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_spmv<L>, dim3(grid_for(m.n * L)), dim3(256), 0, s, m.rowptr, m.colidx,
                       m.vals, m.n, v, b, y);
    return hipGetLastError();
}

// lanes per row: the power of two at or below the mean row length, 1..32
hipError_t launch_csr_spmv(const CsrDev &m, const double *v, const double *b, double *y,
                           hipStream_t s)
{
    const int64_t mean = m.nnz / std::max<int64_t>(m.n, 1);
    if (mean >= 32) return launch_csr_spmv_l<32>(m, v, b, y, s);
    if (mean >= 16) return launch_csr_spmv_l<16>(m, v, b, y, s);
    if (mean >= 8) return launch_csr_spmv_l<8>(m, v, b, y, s);
    if (mean >= 4) return launch_csr_spmv_l<4>(m, v, b, y, s);
    if (mean >= 2) return launch_csr_spmv_l<2>(m, v, b, y, s);
    return launch_csr_spmv_l<1>(m, v, b, y, s);
}

// ------------------------------------------------------------ host stages
namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// Minimum-cost perfect matching of rows to columns.  sigma[i] = column of
// row i; u, v the potentials (c_ij - u_i - v_j >= 0, = 0 on the matching).
// Returns false when A has no perfect matching (structurally singular).
bool db_match(const Csr &c, std::vector<int64_t> &sigma, std::vector<double> &u,
              std::vector<double> &v)
{
    const int64_t n = c.n;
    u.assign(n, kInf);
    v.assign(n, kInf);
    std::vector<int64_t> row_of(n, -1);
    sigma.assign(n, -1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = c.ptr[i]; e < c.ptr[i + 1]; ++e) u[i] = std::min(u[i], c.val[e]);
    for (int64_t i = 0; i < n; ++i) {
        if (u[i] == kInf) return false;                   // an empty row
        for (int64_t e = c.ptr[i]; e < c.ptr[i + 1]; ++e) v[c.col[e]] = std::min(v[c.col[e]], c.val[e] - u[i]);
    }
    for (int64_t j = 0; j < n; ++j)
        if (v[j] == kInf) return false;                   // an empty column
    // initial partial match on tight edges (stage 2 of the paper's DB)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = c.ptr[i]; e < c.ptr[i + 1]; ++e) {
            const int64_t j = c.col[e];
            if (row_of[j] < 0 && c.val[e] - u[i] - v[j] <= 0.0) {
                row_of[j] = i;
                sigma[i] = j;
                break;
            }
        }
    // shortest augmenting paths for the remaining rows (stage 3)
    std::vector<double> d(n, kInf);
    std::vector<int64_t> pred(n, -1);
    std::vector<char> done(n, 0);
    std::vector<int64_t> touched;
    typedef std::pair<double, int64_t> Item;
    for (int64_t f = 0; f < n; ++f) {
        if (sigma[f] >= 0) continue;
        std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
        touched.clear();
        auto relax = [&](int64_t i, double di) {
            for (int64_t e = c.ptr[i]; e < c.ptr[i + 1]; ++e) {
                const int64_t j = c.col[e];
                if (done[j]) continue;
                const double nd = di + (c.val[e] - u[i] - v[j]);
                if (nd < d[j]) {
                    if (d[j] == kInf) touched.push_back(j);
                    d[j] = nd;
                    pred[j] = i;
                    pq.push(Item(nd, j));
                }
            }
        };
        relax(f, 0.0);
        int64_t jstar = -1;
        double dmin = kInf;
        std::vector<int64_t> scanned;
        while (!pq.empty()) {
            const Item it = pq.top();
            pq.pop();
            const int64_t j = it.second;
            if (done[j] || it.first > d[j]) continue;
            done[j] = 1;
            scanned.push_back(j);
            if (row_of[j] < 0) {
                jstar = j;
                dmin = d[j];
                break;
            }
            relax(row_of[j], d[j]);
        }
        if (jstar < 0) return false;                      // no augmenting path
        // potentials: columns finalized before the end move by d_j - dmin
        for (int64_t j : scanned) v[j] += d[j] - dmin;
        // augment along the predecessors
        for (int64_t j = jstar;;) {
            const int64_t i = pred[j];
            const int64_t next = sigma[i];
            sigma[i] = j;
            row_of[j] = i;
            if (i == f) break;
            j = next;
        }
        for (int64_t j : touched) {
            d[j] = kInf;
            pred[j] = -1;
            done[j] = 0;
        }
        // rows: tight on their matched edge
        for (int64_t j : scanned)
            if (row_of[j] >= 0) {
                const int64_t i = row_of[j];
                for (int64_t e = c.ptr[i]; e < c.ptr[i + 1]; ++e)
                    if (c.col[e] == sigma[i]) u[i] = c.val[e] - v[sigma[i]];
            }
        for (int64_t e = c.ptr[f]; e < c.ptr[f + 1]; ++e)
            if (c.col[e] == sigma[f]) u[f] = c.val[e] - v[sigma[f]];
    }
    return true;
}

// Neighbour lists of the structure of B + B^T without self loops, sorted and
// without repeats, as one CSR array (counted, filled, then each list sorted).
struct Adjacency {
    std::vector<int64_t> ptr, idx;
    int64_t degree(int64_t i) const { return ptr[i + 1] - ptr[i]; }
};

Adjacency sym_adjacency(const Csr &b)
{
    const int64_t n = b.n;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = b.ptr[i]; e < b.ptr[i + 1]; ++e) {
            const int64_t j = b.col[e];
            if (j == i) continue;
            ++cnt[i + 1];
            ++cnt[j + 1];
        }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int64_t> raw(cnt[n]), cur(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = b.ptr[i]; e < b.ptr[i + 1]; ++e) {
            const int64_t j = b.col[e];
            if (j == i) continue;
            raw[cur[i]++] = j;
            raw[cur[j]++] = i;
        }
    Adjacency adj;
    adj.ptr.assign(n + 1, 0);
    adj.idx.reserve(raw.size());
    for (int64_t i = 0; i < n; ++i) {
        auto first = raw.begin() + cnt[i], end = raw.begin() + cnt[i + 1];
        std::sort(first, end);
        end = std::unique(first, end);
        adj.idx.insert(adj.idx.end(), first, end);
        adj.ptr[i + 1] = (int64_t)adj.idx.size();
    }
    return adj;
}

int64_t half_bandwidth(const Csr &b, const std::vector<int64_t> &new_of_old)
{
    int64_t k = 0;
    for (int64_t i = 0; i < b.n; ++i)
        for (int64_t e = b.ptr[i]; e < b.ptr[i + 1]; ++e)
            k = std::max<int64_t>(k, std::llabs(new_of_old[i] - new_of_old[b.col[e]]));
    return k;
}

// One Cuthill-McKee ordering (old index by new position) started at s, then
// the other components from their least (degree, index) node; `last`
// receives the last BFS level of s's component.
void cm_from(const Adjacency &adj, const std::vector<int64_t> &deg,
             int64_t s, std::vector<int64_t> &order, std::vector<int64_t> &last)
{
    const int64_t n = (int64_t)deg.size();
    std::vector<char> seen(n, 0);
    std::vector<int64_t> dist(n, -1);
    order.clear();
    auto less = [&](int64_t a, int64_t b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
    auto bfs = [&](int64_t start, bool first) {
        const size_t base = order.size();
        seen[start] = 1;
        dist[start] = 0;
        order.push_back(start);
        std::vector<int64_t> nb;
        for (size_t h = base; h < order.size(); ++h) {
            const int64_t x = order[h];
            nb.clear();
            for (int64_t e = adj.ptr[x]; e < adj.ptr[x + 1]; ++e)
                if (!seen[adj.idx[e]]) nb.push_back(adj.idx[e]);
            std::sort(nb.begin(), nb.end(), less);
            for (int64_t w : nb) {
                seen[w] = 1;
                dist[w] = dist[x] + 1;
                order.push_back(w);
            }
        }
        if (first) {
            int64_t far = 0;
            for (size_t h = base; h < order.size(); ++h) far = std::max(far, dist[order[h]]);
            last.clear();
            for (size_t h = base; h < order.size(); ++h)
                if (dist[order[h]] == far) last.push_back(order[h]);
        }
    };
    bfs(s, true);
    while ((int64_t)order.size() < n) {
        int64_t best = -1;
        for (int64_t v = 0; v < n; ++v)
            if (!seen[v] && (best < 0 || less(v, best))) best = v;
        bfs(best, false);
    }
}

std::vector<int64_t> cuthill_mckee(const Csr &b, int tries)
{
    const int64_t n = b.n;
    const auto adj = sym_adjacency(b);
    std::vector<int64_t> deg(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = adj.degree(i);
    auto less = [&](int64_t a, int64_t c) { return deg[a] != deg[c] ? deg[a] < deg[c] : a < c; };
    int64_t start = 0;
    for (int64_t v = 1; v < n; ++v)
        if (less(v, start)) start = v;
    std::vector<int64_t> best, order, last, tried;
    int64_t best_k = -1;
    for (int t = 0; t < tries; ++t) {
        tried.push_back(start);
        cm_from(adj, deg, start, order, last);
        std::vector<int64_t> new_of_old(n);
        for (int64_t p = 0; p < n; ++p) new_of_old[order[p]] = p;
        const int64_t k = half_bandwidth(b, new_of_old);
        if (best_k < 0 || k < best_k) {
            best = order;
            best_k = k;
        }
        int64_t next = -1;
        for (int64_t x : last)
            if (std::find(tried.begin(), tried.end(), x) == tried.end() && (next < 0 || less(x, next)))
                next = x;
        if (next < 0) break;
        start = next;
    }
    return best;
}

}  // namespace

// The analysis result: maps and scales on the host, the reordered structure
// and the work vectors on the device.
struct SparsePlan {
    int64_t n = 0, nnz = 0;
    int k = 0, k_full = 0;
    std::vector<int32_t> new_row, new_col;    // row r of A -> row of A_hat; column c -> column
    std::vector<double> row_scale, col_scale;
    // the reordered structure: row pointers, columns, source entry and scale
    std::vector<int64_t> h_rowptr, h_src;
    std::vector<int32_t> h_colidx;
    std::vector<double> h_escale;
    // device
    int64_t *rowptr = nullptr;
    int32_t *colidx = nullptr;
    int64_t *src = nullptr;
    double *escale = nullptr, *vals = nullptr;
    int32_t *d_new_row = nullptr, *d_new_col = nullptr;
    double *d_row_scale = nullptr, *d_col_scale = nullptr;
    double *bhat = nullptr, *yhat = nullptr;
    bool assembled = false;
    // host time of the analysis stages (Sec. 3.4 buckets T_DB, T_CM, T_Drop)
    double t_db_ms = 0.0, t_cm_ms = 0.0, t_drop_ms = 0.0;
};

}  // namespace sap

using namespace sap;

struct sap_sparse_ : SparsePlan {};

namespace {

int sfail(int code, const std::string &m) { return api_fail(code, m); }

#define SHIP_TRY(expr)                                                                \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return sfail(SAP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void free_plan(sap_sparse p)
{
    for (void *q : {(void *)p->rowptr, (void *)p->colidx, (void *)p->src, (void *)p->escale,
                    (void *)p->vals, (void *)p->d_new_row, (void *)p->d_new_col,
                    (void *)p->d_row_scale, (void *)p->d_col_scale, (void *)p->bhat, (void *)p->yhat})
        if (q) (void)hipFree(q);
    delete p;
}

}  // namespace

extern "C" {

int sap_sparse_create(int64_t n, const int64_t *rowptr, const int32_t *colidx, const double *vals,
                      int32_t db, int32_t cm, double drop_frac, sap_sparse *out)
{
    if (!out) return sfail(SAP_ERR_INVALID, "output pointer is null");
    *out = nullptr;
    if (n < 1 || n > INT32_MAX || !rowptr || !colidx || !vals)
        return sfail(SAP_ERR_INVALID, "bad CSR arguments");
    if (!(drop_frac >= 0.0 && drop_frac < 1.0)) return sfail(SAP_ERR_INVALID, "drop_frac must be in [0, 1)");
    if (rowptr[0] != 0) return sfail(SAP_ERR_INVALID, "rowptr[0] must be 0");
    Csr a;
    a.n = n;
    a.ptr.assign(rowptr, rowptr + n + 1);
    const int64_t nnz = a.ptr[n];
    for (int64_t i = 0; i < n; ++i)
        if (a.ptr[i + 1] < a.ptr[i]) return sfail(SAP_ERR_INVALID, "rowptr must not decrease");
    a.col.assign(colidx, colidx + nnz);
    a.val.assign(vals, vals + nnz);
    for (int64_t e = 0; e < nnz; ++e)
        if (a.col[e] < 0 || a.col[e] >= n) return sfail(SAP_ERR_INVALID, "column index out of range");
    for (int64_t e = 0; e < nnz; ++e)
        if (!std::isfinite(a.val[e])) return sfail(SAP_ERR_INVALID, "a value is not finite");
    {
        // a repeated (row, column) would be summed by the product but not by the band
        std::vector<int64_t> last(n, -1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = a.ptr[i]; e < a.ptr[i + 1]; ++e) {
                if (last[a.col[e]] == i) return sfail(SAP_ERR_INVALID, "a column repeats within a row");
                last[a.col[e]] = i;
            }
    }

    sap_sparse p = new (std::nothrow) sap_sparse_();
    if (!p) return sfail(SAP_ERR_INVALID, "out of host memory");
    p->n = n;
    p->nnz = nnz;
    using clk = std::chrono::steady_clock;
    auto ms_since = [](clk::time_point t0) {
        return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    };
    auto t0 = clk::now();
    // DB: costs c_ij = log a_i - log|a_ij| (explicit zeros are not edges)
    std::vector<int64_t> sigma(n);
    std::vector<double> rs(n, 1.0), cs(n, 1.0);
    if (db) {
        Csr c;
        c.n = n;
        c.ptr.assign(n + 1, 0);
        std::vector<double> amax(n, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = a.ptr[i]; e < a.ptr[i + 1]; ++e) amax[i] = std::max(amax[i], std::fabs(a.val[e]));
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t e = a.ptr[i]; e < a.ptr[i + 1]; ++e)
                if (a.val[e] != 0.0) {
                    c.col.push_back(a.col[e]);
                    c.val.push_back(std::log(amax[i]) - std::log(std::fabs(a.val[e])));
                }
            c.ptr[i + 1] = (int64_t)c.col.size();
        }
        std::vector<double> u, v;
        if (!db_match(c, sigma, u, v)) {
            delete p;
            return sfail(SAP_ERR_SINGULAR, "A is structurally singular (no perfect matching)");
        }
        for (int64_t i = 0; i < n; ++i) {
            rs[i] = std::exp(u[i]) / amax[i];
            cs[i] = std::exp(v[i]);
        }
    } else {
        std::iota(sigma.begin(), sigma.end(), 0);
    }
    p->t_db_ms = ms_since(t0);
    t0 = clk::now();
    // B = Q A: row i of A becomes row sigma[i]
    Csr b;
    b.n = n;
    {
        std::vector<int64_t> cnt(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) cnt[sigma[i] + 1] = a.ptr[i + 1] - a.ptr[i];
        for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
        b.ptr = cnt;
        b.col.resize(nnz);
        for (int64_t i = 0; i < n; ++i)
            std::copy(a.col.begin() + a.ptr[i], a.col.begin() + a.ptr[i + 1], b.col.begin() + b.ptr[sigma[i]]);
    }
    // CM on B + B^T
    std::vector<int64_t> pos(n);
    if (cm) {
        const std::vector<int64_t> order = cuthill_mckee(b, 3);
        for (int64_t q = 0; q < n; ++q) pos[order[q]] = q;
    } else {
        std::iota(pos.begin(), pos.end(), 0);
    }
    p->new_row.resize(n);
    p->new_col.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        p->new_row[i] = (int32_t)pos[sigma[i]];
        p->new_col[i] = (int32_t)pos[i];
    }
    p->t_cm_ms = ms_since(t0);
    t0 = clk::now();
    p->row_scale = rs;
    p->col_scale = cs;
    // the reordered structure, entries sorted by (row, column) of A_hat
    // (rows of A_hat by counting, then each row's few entries by column; the
    // keys are unique since no column repeats within a row)
    std::vector<int64_t> ent(nnz), erow(nnz);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = a.ptr[i]; e < a.ptr[i + 1]; ++e) erow[e] = i;
    {
        std::vector<int64_t> cur(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) cur[p->new_row[i] + 1] = a.ptr[i + 1] - a.ptr[i];
        for (int64_t r = 0; r < n; ++r) cur[r + 1] += cur[r];
        for (int64_t e = 0; e < nnz; ++e) ent[cur[p->new_row[erow[e]]]++] = e;
        int64_t lo = 0;
        for (int64_t r = 0; r < n; ++r) {
            const int64_t hi = cur[r];          // end of row r after the fill
            std::sort(ent.begin() + lo, ent.begin() + hi, [&](int64_t x, int64_t y) {
                return p->new_col[a.col[x]] < p->new_col[a.col[y]];
            });
            lo = hi;
        }
    }
    std::vector<int64_t> hptr(n + 1, 0);
    std::vector<int32_t> hcol(nnz);
    std::vector<double> hscale(nnz);
    int64_t kfull = 0;
    std::vector<double> per_off;      // |a_hat| mass per distance from the diagonal
    for (int64_t q = 0; q < nnz; ++q) {
        const int64_t e = ent[q];
        const int32_t r = p->new_row[erow[e]], c = p->new_col[a.col[e]];
        hptr[r + 1] += 1;
        hcol[q] = c;
        hscale[q] = rs[erow[e]] * cs[a.col[e]];
        const int64_t off = std::llabs((int64_t)r - c);
        kfull = std::max(kfull, off);
        if ((int64_t)per_off.size() <= off) per_off.resize(off + 1, 0.0);
        per_off[off] += std::fabs(a.val[e] * hscale[q]);
    }
    for (int64_t i = 0; i < n; ++i) hptr[i + 1] += hptr[i];
    // drop-off: least K whose outside entries carry <= drop_frac of the total
    double total = 0.0;
    for (double m : per_off) total += m;
    int64_t k = kfull;
    double tail = 0.0;                 // mass beyond the candidate K
    for (int64_t kk = kfull; kk >= 0; --kk) {
        if (tail <= drop_frac * total) k = kk;
        else break;
        tail += per_off[kk];
    }
    p->k_full = (int)kfull;
    p->k = (int)k;
    p->h_rowptr = std::move(hptr);
    p->h_colidx = std::move(hcol);
    p->h_src = std::move(ent);
    p->h_escale = std::move(hscale);
    p->t_drop_ms = ms_since(t0);
    *out = p;
    return SAP_OK;
}

// device copies of the plan, made by the first sap_sparse_assemble (the
// analysis itself touches no device)
static int upload_plan(sap_sparse p)
{
    if (p->rowptr) return SAP_OK;
    auto up = [&](auto *&dst, const auto &vec) -> hipError_t {
        using E = typename std::decay<decltype(vec[0])>::type;
        hipError_t e = hipMalloc((void **)&dst, sizeof(E) * std::max<size_t>(vec.size(), 1));
        if (e != hipSuccess) return e;
        return hipMemcpy(dst, vec.data(), sizeof(E) * vec.size(), hipMemcpyHostToDevice);
    };
    hipError_t e = up(p->rowptr, p->h_rowptr);
    if (e == hipSuccess) e = up(p->colidx, p->h_colidx);
    if (e == hipSuccess) e = up(p->src, p->h_src);
    if (e == hipSuccess) e = up(p->escale, p->h_escale);
    if (e == hipSuccess) e = up(p->d_new_row, p->new_row);
    if (e == hipSuccess) e = up(p->d_new_col, p->new_col);
    if (e == hipSuccess) e = up(p->d_row_scale, p->row_scale);
    if (e == hipSuccess) e = up(p->d_col_scale, p->col_scale);
    if (e == hipSuccess) e = hipMalloc((void **)&p->vals, sizeof(double) * std::max<int64_t>(p->nnz, 1));
    if (e == hipSuccess) e = hipMalloc((void **)&p->bhat, sizeof(double) * p->n);
    if (e == hipSuccess) e = hipMalloc((void **)&p->yhat, sizeof(double) * p->n);
    if (e != hipSuccess) return sfail(SAP_ERR_HIP, std::string("sparse plan upload: ") + hipGetErrorString(e));
    return SAP_OK;
}

int sap_sparse_info(sap_sparse p, int32_t *k, int32_t *k_full, int32_t *new_row, int32_t *new_col,
                    double *row_scale, double *col_scale)
{
    if (!p) return sfail(SAP_ERR_INVALID, "null plan");
    if (k) *k = p->k;
    if (k_full) *k_full = p->k_full;
    if (new_row) std::copy(p->new_row.begin(), p->new_row.end(), new_row);
    if (new_col) std::copy(p->new_col.begin(), p->new_col.end(), new_col);
    if (row_scale) std::copy(p->row_scale.begin(), p->row_scale.end(), row_scale);
    if (col_scale) std::copy(p->col_scale.begin(), p->col_scale.end(), col_scale);
    return SAP_OK;
}

int sap_sparse_times(sap_sparse p, double *t_db_ms, double *t_cm_ms, double *t_drop_ms)
{
    if (!p) return sfail(SAP_ERR_INVALID, "null plan");
    if (t_db_ms) *t_db_ms = p->t_db_ms;
    if (t_cm_ms) *t_cm_ms = p->t_cm_ms;
    if (t_drop_ms) *t_drop_ms = p->t_drop_ms;
    return SAP_OK;
}

int sap_sparse_assemble(sap_sparse p, const double *vals, double *band, void *stream)
{
    if (!p) return sfail(SAP_ERR_INVALID, "null plan");
    if (!vals || !band) return sfail(SAP_ERR_INVALID, "null pointer");
    if (const int rc = upload_plan(p)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_sparse_values, dim3(grid_for(p->nnz)), dim3(256), 0, s, vals, p->src,
                       p->escale, p->vals, p->nnz);
    SHIP_TRY(hipGetLastError());
    SHIP_TRY(launch_fill(band, 0.0, (int64_t)(2 * p->k + 1) * p->n, s));
    hipLaunchKernelGGL(k_band_from_csr, dim3(grid_for(p->n)), dim3(256), 0, s, p->rowptr, p->colidx,
                       p->vals, p->n, p->k, band);
    SHIP_TRY(hipGetLastError());
    p->assembled = true;
    return SAP_OK;
}

int sap_sparse_destroy(sap_sparse p)
{
    if (p) free_plan(p);
    return SAP_OK;
}

}  // extern "C"

namespace sap {

// pieces sap_solve_sparse needs from the plan (sap_api.hip)
bool sparse_plan_parts(sap_sparse p, CsrDev *m, double **bhat, double **yhat,
                       const int32_t **new_row, const int32_t **new_col, const double **rs,
                       const double **cs)
{
    if (!p || !p->assembled) return false;
    m->n = p->n;
    m->nnz = p->nnz;
    m->rowptr = p->rowptr;
    m->colidx = p->colidx;
    m->vals = p->vals;
    *bhat = p->bhat;
    *yhat = p->yhat;
    *new_row = p->d_new_row;
    *new_col = p->d_new_col;
    *rs = p->d_row_scale;
    *cs = p->d_col_scale;
    return true;
}

int sparse_plan_k(sap_sparse p) { return p ? p->k : -1; }

hipError_t launch_map_vec(const double *in, const int32_t *map, const double *scale, double *out,
                          int64_t n, int gather, hipStream_t s)
{
    hipLaunchKernelGGL(k_map_vec, dim3(grid_for(n)), dim3(256), 0, s, in, map, scale, out, n, gather);
    return hipGetLastError();
}

}  // namespace sap
