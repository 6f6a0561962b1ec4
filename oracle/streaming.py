"""Streaming extension (Sec. III-D), oracle side.  Test infrastructure: only
tests, the smoke check and the benchmark's CPU baseline use it.

When a set E' of new edges arrives, only the endpoints V' of E' change
degree.  For the NCut operator M (Eq. 2), M_ij depends on A_ij, d_i and d_j
alone, so M changes only in the rows and columns of V'; the same holds for
the GCN operator of Eq. 6.  Level t of the projection, Y_t = X Y_{t-1}
(Y_0 = Theta), can therefore change only on the nodes within t hops of V' in
the new graph, and GCN layer k only within q + k hops; the union of these
balls is V' together with its multi-hop neighbourhood V''.  The incremental
update recomputes every level on its ball only, from the current values of
the level below, so its cost follows the edges E'' incident to the balls.

Readings (the section states the idea, not the procedure):
* E' adds undirected edges between existing nodes; an edge already in the
  graph, a repeated new edge or a self pair is an error, and no node is
  added;
* the update is local for X = M only.  The modularity operators (Eq. 4 and
  the reduced Q~) carry the factor 1/2e in every entry, and any new edge
  changes 2e, so for them every row of every level is recomputed (the ball
  is all of V); the tests below pin that these levels do change outside the
  hop balls;
* the levels kept between updates are Theta, Y_1..Y_q, the input of layer 1
  (Y_q, or its row-normalised copy when the input is normalised) and the
  outputs H_1..H_n of the layers (H_n = Z);
* k-means and model selection run again on the updated embedding; they are
  not incremental here.

Pinned in ``tests/test_oracle_streaming.py``: the update equals a full
recomputation on the new graph (the projection levels bit for bit), levels
outside their hop balls are unchanged between the old and new graph under M
(and change under the modularity operators), hop distances equal
``scipy.sparse.csgraph`` shortest paths, and the merged CSR is valid.
"""
import numpy as np
from scipy.sparse import csgraph

from . import gcn, projection
from .graph import adjacency, degrees, two_e


def add_edges(row_ptr, col_idx, n, src, dst):
    """CSR of the graph with the undirected edges (src[e], dst[e]) added.
    Raises ValueError on a self pair, an edge out of range, a repeated new
    edge or an edge already present."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    if np.any(src < 0) or np.any(src >= n) or np.any(dst < 0) or np.any(dst >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(src == dst):
        raise ValueError("self pair")
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    old_rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    old_key = old_rows * n + col_idx
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    new_key = np.concatenate([lo * n + hi, hi * n + lo])
    if np.unique(new_key).size != new_key.size:
        raise ValueError("repeated new edge")
    if np.intersect1d(old_key, new_key).size:
        raise ValueError("edge already present")
    key = np.sort(np.concatenate([old_key, new_key]))
    rows, cols = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols


def hop_distance(row_ptr, col_idx, n, sources, radius):
    """Hops from the nearest node of `sources`, radius + 1 for every node
    farther than `radius` (breadth-first, level by level)."""
    dist = np.full(n, radius + 1, dtype=np.int64)
    frontier = np.unique(np.asarray(sources, dtype=np.int64))
    dist[frontier] = 0
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    for t in range(1, radius + 1):
        if frontier.size == 0:
            break
        nb = np.concatenate([col_idx[row_ptr[i]:row_ptr[i + 1]] for i in frontier])
        nb = np.unique(nb)
        nb = nb[dist[nb] > t]
        dist[nb] = t
        frontier = nb
    return dist


def hop_distance_library(row_ptr, col_idx, n, sources, radius):
    """The same distances from scipy's unweighted shortest paths."""
    a = adjacency(row_ptr, col_idx, n)
    d = csgraph.shortest_path(a, unweighted=True, indices=np.unique(sources))
    d = np.min(np.atleast_2d(d), axis=0)
    out = np.where(np.isfinite(d), d, radius + 1).astype(np.int64)
    return np.minimum(out, radius + 1)


def _operator(row_ptr, col_idx, n, op):
    if op == projection.NCUT:
        return projection.ncut_operator(row_ptr, col_idx, n).tocsr()
    if op == projection.MOD_REDUCED:
        return projection.reduced_modularity_operator(row_ptr, col_idx, n).tocsr()
    return None


def _step(row_ptr, col_idx, n, op, y, rows=None):
    """Rows `rows` (all when None) of X y."""
    if op == projection.MOD_FULL:
        a = adjacency(row_ptr, col_idx, n)
        d = degrees(row_ptr).astype(np.float64)
        full = projection.apply_modularity(a, d, float(two_e(row_ptr)), y)
        return full if rows is None else full[rows]
    x = _operator(row_ptr, col_idx, n, op)
    return x @ y if rows is None else x[rows] @ y


def levels(row_ptr, col_idx, n, op, L, q, dims, seed, normalize_input=False):
    """Every level of the embedding of one graph: {'y': [Theta, Y_1..Y_q],
    'h0': input of layer 1, 'h': [H_1..H_n]} (FP64)."""
    y = [projection.theta(seed, n, L)]
    for _ in range(q):
        y.append(np.asarray(_step(row_ptr, col_idx, n, op, y[-1])))
    h0 = gcn.row_normalize(y[-1]) if normalize_input else y[-1].copy()
    ahat = gcn.gcn_operator(row_ptr, col_idx, n)
    h, cur, l_in = [], h0, L
    for k, l_out in enumerate(dims, start=1):
        w = gcn.weight(seed, k, l_in, l_out)
        cur = gcn.row_normalize(np.tanh((ahat @ cur) @ w))
        h.append(cur)
        l_in = l_out
    return {"y": y, "h0": h0, "h": h}


def update(prev, row_ptr, col_idx, n, op, q, dims, seed, vprime, normalize_input=False):
    """Levels of the new graph (row_ptr, col_idx) from the previous graph's
    levels `prev`: every level recomputed on its hop ball around `vprime`
    (all rows for the modularity operators).  Returns (levels, sizes) with
    sizes[t - 1] = rows recomputed at level t (t = 1..q + len(dims))."""
    radius = q + len(dims)
    if op == projection.NCUT:
        dist = hop_distance(row_ptr, col_idx, n, vprime, radius)
    else:
        dist = np.zeros(n, dtype=np.int64)
    y = [lv.copy() for lv in prev["y"]]
    sizes = []
    for t in range(1, q + 1):
        rows = np.flatnonzero(dist <= t)
        y[t][rows] = _step(row_ptr, col_idx, n, op, y[t - 1], rows)
        sizes.append(rows.size)
    h0 = prev["h0"].copy()
    rows = np.flatnonzero(dist <= q)
    h0[rows] = gcn.row_normalize(y[q][rows]) if normalize_input else y[q][rows]
    ahat = gcn.gcn_operator(row_ptr, col_idx, n)
    h, cur, l_in = [], h0, h0.shape[1]
    for k, l_out in enumerate(dims, start=1):
        rows = np.flatnonzero(dist <= q + k)
        w = gcn.weight(seed, k, l_in, l_out)
        nxt = prev["h"][k - 1].copy()
        nxt[rows] = gcn.row_normalize(np.tanh((ahat[rows] @ cur) @ w))
        h.append(nxt)
        sizes.append(rows.size)
        cur, l_in = nxt, l_out
    return {"y": y, "h0": h0, "h": h}, sizes
