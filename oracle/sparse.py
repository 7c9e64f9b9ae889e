"""Sparse front end of SaP, CPU oracle -- TEST INFRASTRUCTURE ONLY.

The reorderings that turn a sparse A into the dense banded matrix the SaP
preconditioner is built on (paper: Li, Serban, Negrut, arXiv:1509.07919):

* ``db_cost`` / ``db_matching`` -- diagonal boosting (Sec. 3.1, "Diagonal
  Boosting"): a row permutation maximising prod |a_{i sigma_i}|, as the
  minimum-cost perfect bipartite matching with costs
  c_ij = log a_i - log |a_ij|, a_i = max_j |a_ij| (eq:DBrelated), found
  by successive shortest augmenting paths (the Hungarian method with
  Dijkstra's algorithm on reduced costs; Kuhn 1955, Edmonds-Karp 1972),
  whose dual potentials u, v give the I-matrix scaling
  exp(u_i)/a_i, exp(v_j).  Pinned against brute force on small matrices
  and against SciPy's min_weight_full_bipartite_matching (a library
  routine, fast on some inputs and not on others, so only the former).
* ``cuthill_mckee`` -- bandwidth reduction (Sec. 3.1, "Bandwidth
  reduction"; Sec. 3.3): Cuthill-McKee on the structure of B + B^T, a
  breadth-first search that visits the neighbours of each node in
  ascending degree, started from several nodes, keeping the ordering with
  the smallest half-bandwidth.  Deterministic tie-breaks (degree, then
  index) make the ordering unique.
* ``drop_k`` -- element drop-off (Sec. 3.4, T_Drop): the smallest
  half-bandwidth K whose outside-the-band entries carry at most a fraction
  ``frac`` of sum |a_ij|.
"""

from __future__ import annotations

import heapq

import numpy as np
import scipy.sparse as sps
from scipy.sparse.csgraph import min_weight_full_bipartite_matching


def _csr(n, rowptr, colidx, vals):
    return sps.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colidx),
                           np.asarray(rowptr)), shape=(n, n))


def db_costs(n, rowptr, colidx, vals) -> sps.csr_matrix:
    """c_ij = log a_i - log|a_ij| on the nonzeros (eq:DBrelated); >= 0, and 0
    for the largest entry of each row."""
    A = _csr(n, rowptr, colidx, vals)
    absA = abs(A)
    amax = np.asarray(absA.max(axis=1).todense()).ravel()
    C = absA.copy().tocsr()
    rows = np.repeat(np.arange(n), np.diff(C.indptr))
    C.data = np.log(amax[rows]) - np.log(C.data)
    return C


def db_matching(n, rowptr, colidx, vals):
    """sigma[i] = column matched to row i in a minimum-cost perfect matching,
    and that minimum cost sum_i c_{i sigma_i}.  (sigma, cost, u, v) with
    ``duals=True`` via db_matching_duals."""
    sigma, cost, _, _ = db_matching_duals(n, rowptr, colidx, vals)
    return sigma, cost


def db_matching_duals(n, rowptr, colidx, vals):
    """Minimum-cost perfect matching by successive shortest augmenting paths.

    Dual feasibility: reduced costs r_ij = c_ij - u_i - v_j >= 0 on every
    edge, = 0 on matched edges (then the matching is optimal).  Start:
    v_j = min_i c_ij, u_i = min_j (c_ij - v_j), and each row takes a free
    column of zero reduced cost if it has one.  For every row i0 still
    free: Dijkstra from i0 over alternating paths (row -> column along an
    edge, length r_ij; column -> its matched row, length 0) until the
    nearest free column j* is popped, at distance L; augment along the path;
    every row i reached at distance d_i gets u_i += L - d_i and every column
    j popped at distance d_j gets v_j -= L - d_j, which keeps r >= 0 and
    makes the new path's edges tight.  Raises ValueError if A has no
    perfect matching (structurally singular)."""
    C = db_costs(n, rowptr, colidx, vals)
    ptr, col, cost = C.indptr, C.indices, C.data
    inf = float("inf")
    v = np.full(n, inf)
    for i in range(n):
        for e in range(ptr[i], ptr[i + 1]):
            v[col[e]] = min(v[col[e]], cost[e])
    if np.isinf(v).any():
        raise ValueError("structurally singular: an empty column")
    u = np.zeros(n)
    row_of = np.full(n, -1, dtype=np.int64)        # column -> matched row
    sigma = np.full(n, -1, dtype=np.int64)         # row -> matched column
    for i in range(n):
        if ptr[i] == ptr[i + 1]:
            raise ValueError("structurally singular: an empty row")
        u[i] = min(cost[e] - v[col[e]] for e in range(ptr[i], ptr[i + 1]))
        for e in range(ptr[i], ptr[i + 1]):
            j = col[e]
            if row_of[j] < 0 and cost[e] - v[j] - u[i] == 0.0:
                row_of[j], sigma[i] = i, j
                break
    for i0 in range(n):
        if sigma[i0] >= 0:
            continue
        dist = {}                  # column -> tentative distance
        via = {}                   # column -> row it was reached from
        done = {}                  # column -> final distance
        rows = {i0: 0.0}           # rows reached -> their distance
        heap = []
        i, di = i0, 0.0
        jstar = -1
        while True:
            for e in range(ptr[i], ptr[i + 1]):
                j = col[e]
                if j in done:
                    continue
                nd = di + (cost[e] - u[i] - v[j])
                if nd < dist.get(j, inf):
                    dist[j], via[j] = nd, i
                    heapq.heappush(heap, (nd, j))
            while heap and (heap[0][1] in done or heap[0][0] > dist[heap[0][1]]):
                heapq.heappop(heap)
            if not heap:
                raise ValueError("structurally singular: no augmenting path")
            dj, j = heapq.heappop(heap)
            done[j] = dj
            if row_of[j] < 0:
                jstar, L = j, dj
                break
            i, di = row_of[j], dj
            rows[i] = di
        for i, di in rows.items():
            u[i] += L - di
        for j, dj in done.items():
            v[j] -= L - dj
        j = jstar
        while True:                # flip the path back to i0
            i = via[j]
            nxt = sigma[i]
            sigma[i], row_of[j] = j, i
            if i == i0:
                break
            j = nxt
    total = float(sum(C[i, sigma[i]] for i in range(n)))
    return sigma, total, u, v


def db_matching_scipy(n, rowptr, colidx, vals):
    """The same optimum from SciPy's min_weight_full_bipartite_matching
    (edge weights shifted by +1 so that zero costs stay edges)."""
    C = db_costs(n, rowptr, colidx, vals)
    W = C.copy()
    W.data = W.data + 1.0
    r, c = min_weight_full_bipartite_matching(W)
    sigma = np.empty(n, dtype=np.int64)
    sigma[r] = c
    return sigma, float(sum(C[i, sigma[i]] for i in range(n)))


def matching_cost(n, rowptr, colidx, vals, sigma) -> float:
    C = db_costs(n, rowptr, colidx, vals)
    return float(sum(C[i, int(sigma[i])] for i in range(n)))


def _sym_adjacency(n, rowptr, colidx):
    """Neighbour lists of the structure of B + B^T (no self loops), sorted."""
    B = sps.csr_matrix((np.ones(len(colidx)), np.asarray(colidx), np.asarray(rowptr)), shape=(n, n))
    S = (B + B.T).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    S.sort_indices()
    return [S.indices[S.indptr[i]:S.indptr[i + 1]].tolist() for i in range(n)]


def _cm_from(adj, deg, start, n):
    """One Cuthill-McKee ordering of the component of `start`, then of the
    remaining components (each from its minimum-(degree, index) node)."""
    order, seen = [], np.zeros(n, dtype=bool)
    levels_last = []

    def bfs(s):
        nonlocal levels_last
        seen[s] = True
        q = [s]
        lev = [s]
        head = 0
        last = [s]
        while head < len(q):
            v = q[head]
            head += 1
            nb = [w for w in adj[v] if not seen[w]]
            nb.sort(key=lambda w: (deg[w], w))
            for w in nb:
                seen[w] = True
                q.append(w)
        order.extend(q)
        # the last BFS level of this component (for the next start)
        dist = {s: 0}
        for v in q:
            for w in adj[v]:
                if w not in dist:
                    dist[w] = dist[v] + 1
        far = max(dist.values())
        levels_last = [v for v in q if dist[v] == far]

    bfs(start)
    first_last = levels_last
    while len(order) < n:
        rest = [v for v in range(n) if not seen[v]]
        bfs(min(rest, key=lambda v: (deg[v], v)))
    return np.array(order, dtype=np.int64), first_last


def half_bandwidth(n, rowptr, colidx, new_of_old) -> int:
    """max |p(r) - p(c)| over the nonzeros, p = new_of_old."""
    rows = np.repeat(np.arange(n), np.diff(np.asarray(rowptr)))
    p = np.asarray(new_of_old)
    if len(rows) == 0:
        return 0
    return int(np.abs(p[rows] - p[np.asarray(colidx)]).max())


def cuthill_mckee(n, rowptr, colidx, tries: int = 3):
    """old_of_new ordering (new index -> old index) and its half-bandwidth.
    Start from the node of least (degree, index); each further try starts
    from the least-(degree, index) node of the previous try's last BFS level
    not tried before; the first ordering of least half-bandwidth wins."""
    adj = _sym_adjacency(n, rowptr, colidx)
    deg = np.array([len(a) for a in adj])
    start = int(min(range(n), key=lambda v: (deg[v], v)))
    tried, best, best_k = set(), None, None
    for _ in range(tries):
        tried.add(start)
        order, last = _cm_from(adj, deg, start, n)
        new_of_old = np.empty(n, dtype=np.int64)
        new_of_old[order] = np.arange(n)
        k = half_bandwidth(n, rowptr, colidx, new_of_old)
        if best is None or k < best_k:
            best, best_k = order, k
        cand = [v for v in last if v not in tried]
        if not cand:
            break
        start = int(min(cand, key=lambda v: (deg[v], v)))
    return best, best_k


def drop_k(n, rowptr, colidx, vals, frac: float) -> int:
    """Smallest K such that the entries with |r - c| > K carry at most
    frac * sum|a| (frac = 0: the half-bandwidth itself)."""
    rows = np.repeat(np.arange(n), np.diff(np.asarray(rowptr)))
    off = np.abs(rows - np.asarray(colidx))
    mass = np.abs(np.asarray(vals))
    kmax = int(off.max()) if len(off) else 0
    per = np.bincount(off, weights=mass, minlength=kmax + 1)
    total = mass.sum()
    # dropped(K) = sum_{d > K} per[d]
    tail = np.concatenate([np.cumsum(per[::-1])[::-1][1:], [0.0]])
    for k in range(kmax + 1):
        if tail[k] <= frac * total:
            return k
    return kmax


def permute_csr(n, rowptr, colidx, vals, new_row, new_col, row_scale=None, col_scale=None):
    """CSR of B with b[new_row[r], new_col[c]] = rs[r] a[r, c] cs[c]."""
    A = _csr(n, rowptr, colidx, vals).tocoo()
    rs = np.ones(n) if row_scale is None else np.asarray(row_scale)
    cs = np.ones(n) if col_scale is None else np.asarray(col_scale)
    B = sps.csr_matrix((rs[A.row] * A.data * cs[A.col], (np.asarray(new_row)[A.row],
                                                          np.asarray(new_col)[A.col])), shape=(n, n))
    B.sort_indices()
    return B
