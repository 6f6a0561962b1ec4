"""Degree-corrected stochastic block model graphs (input generation).

The generative model is the paper's SBM definition (Sec. II): entries
A_ij ~ Pois(theta_i theta_j Omega_{c_i c_j}) independently per node pair, with
counts collapsed to 1 (unweighted graph) and no self-pairs.  The paper's
Alg. 2 samples exactly this distribution by skip-sampling along each block
pair.  This module samples the same exact distribution by Poisson splitting
instead, which vectorises in NumPy: within block pair (r, s) the total count is
Poisson with mean sum_{i in r, j in s} lambda_ij, and each event picks its
endpoints independently with probability proportional to theta.  (Both give
independent Pois(lambda_ij) counts per pair.)

Parameterisation (matching the workload descriptions):
  * block sizes: Dirichlet(alpha) proportions, largest-remainder rounding to N
    with a floor of ``min_block`` nodes;
  * expected degrees: truncated continuous power law ~ d^-gamma on
    [d_min, d_max], by inverse CDF;
  * Omega: off-diagonal Omega_rs = beta vol_r vol_s / V, diagonal fills each
    block's volume, with beta chosen so expected intra/inter edge ratio = rho;
  * node ids randomly permuted so blocks are not contiguous.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray      # int32 [n+1]
    col_idx: np.ndarray      # int32 [nnz]
    planted: np.ndarray      # int32 [n] planted block ids (may be empty)
    info: dict

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def edges_to_csr(n, src, dst):
    """Symmetric, sorted, duplicate- and loop-free CSR from an edge list."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.concatenate([src * n + dst, dst * n + src])
    key = np.unique(key)
    rows = key // n
    cols = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("graph too large for int32 CSR")
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def hub_graph(seed, n=3001, hubs=12):
    """Sparse uniform edges (six per node) plus `hubs` hub nodes joined to
    0.6 % .. 97 % of the nodes: rows of up to ~0.97 n entries next to rows of
    a few.  Returns (row_ptr, col_idx)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, 6 * n)
    dst = rng.integers(0, n, 6 * n)
    centres = rng.choice(n, hubs, replace=False)
    for h, frac in zip(centres, np.linspace(0.006, 0.97, hubs)):
        nb = rng.choice(n, int(frac * n), replace=False)
        src = np.concatenate([src, np.full(nb.size, h)])
        dst = np.concatenate([dst, nb])
    return edges_to_csr(n, src, dst)


def _block_sizes(rng, n, k, alpha, min_block):
    p = rng.dirichlet(np.full(k, alpha))
    raw = n * p
    sizes = np.floor(raw).astype(np.int64)
    rem = n - sizes.sum()
    order = np.argsort(-(raw - sizes), kind="stable")
    sizes[order[:rem]] += 1
    # floor of min_block nodes, deficit taken from the largest blocks
    while sizes.min() < min_block:
        i = int(np.argmin(sizes))
        j = int(np.argmax(sizes))
        need = min_block - sizes[i]
        give = min(need, sizes[j] - min_block)
        if give <= 0:
            raise ValueError("cannot satisfy the minimum block size")
        sizes[i] += give
        sizes[j] -= give
    return sizes


def _power_law(rng, size, gamma, d_min, d_max):
    u = rng.random(size)
    a = 1.0 - gamma
    lo, hi = d_min ** a, d_max ** a
    return (lo + u * (hi - lo)) ** (1.0 / a)


def sample_edges(rng, theta, omega, sizes):
    """Edges (i < j not guaranteed; i != j) of one draw of the Poisson SBM with
    nodes grouped by block (block r = nodes start[r]..start[r+1]-1), theta
    summing to 1 within each block, and block matrix omega.  Multi-edges may
    repeat; the caller collapses them."""
    k = sizes.size
    block_of = np.repeat(np.arange(k), sizes)
    start = np.concatenate([[0], np.cumsum(sizes)])
    cum = np.cumsum(theta)                              # block r spans (r, r+1]
    sq = np.bincount(block_of, weights=theta * theta, minlength=k)

    def draw(blocks):
        u = rng.random(blocks.size)
        pos = np.searchsorted(cum, blocks + u, side="right")
        return np.clip(pos, start[blocks], start[blocks + 1] - 1)

    iu, ju = np.triu_indices(k, 1)
    cnt = rng.poisson(omega[iu, ju])                    # sum theta = 1 per block
    r = np.repeat(iu, cnt)
    s = np.repeat(ju, cnt)
    src = [draw(r)]
    dst = [draw(s)]
    # diagonal: unordered pairs i<j, total mean Omega_rr (1 - sum theta^2) / 2
    cnt = rng.poisson(np.diag(omega) * (1.0 - sq) / 2.0)
    r = np.repeat(np.arange(k), cnt)
    a = draw(r)
    b = draw(r)
    bad = a == b
    while np.any(bad):                                  # condition on i != j
        b[bad] = draw(r[bad])
        bad = a == b
    src.append(a)
    dst.append(b)
    return np.concatenate(src), np.concatenate(dst)


def dcsbm_model(n, k, alpha=2.0, gamma=2.5, d_min=10.0, d_max=100.0, rho=2.5,
                seed=0, min_block=10):
    """The parameters of a DC-SBM graph with the recipe of ``dcsbm`` and no
    sampling: (theta [n] FP64, blocks [n] int32, omega [k x k] FP64), node
    ids randomly permuted, for samplers that take the model itself."""
    rng = np.random.default_rng(np.random.SeedSequence([0x5C, int(seed)]))
    sizes = _block_sizes(rng, n, k, alpha, min_block)
    block_of = np.repeat(np.arange(k), sizes)
    tdeg = _power_law(rng, n, gamma, d_min, d_max)
    vol = np.bincount(block_of, weights=tdeg, minlength=k)
    V = vol.sum()
    S = V - np.sum(vol * vol) / V
    beta = V / ((1.0 + rho) * S)
    omega = beta * np.outer(vol, vol) / V
    np.fill_diagonal(omega, 0.0)
    diag = vol - omega.sum(axis=1)
    if np.any(diag < 0):
        raise ValueError("intra/inter ratio infeasible for these block volumes")
    np.fill_diagonal(omega, diag)
    theta = tdeg / vol[block_of]
    perm = rng.permutation(n)
    theta_p = np.empty(n)
    blocks_p = np.empty(n, dtype=np.int32)
    theta_p[perm] = theta
    blocks_p[perm] = block_of
    return theta_p, blocks_p, omega


def dcsbm(n, k, alpha=2.0, gamma=2.5, d_min=10.0, d_max=100.0, rho=2.5,
          seed=0, min_block=10):
    rng = np.random.default_rng(np.random.SeedSequence([0x5B, int(seed)]))
    sizes = _block_sizes(rng, n, k, alpha, min_block)
    block_of = np.repeat(np.arange(k), sizes)          # nodes grouped by block
    start = np.concatenate([[0], np.cumsum(sizes)])
    tdeg = _power_law(rng, n, gamma, d_min, d_max)
    vol = np.bincount(block_of, weights=tdeg, minlength=k)
    V = vol.sum()
    S = V - np.sum(vol * vol) / V
    beta = V / ((1.0 + rho) * S)
    omega = beta * np.outer(vol, vol) / V
    np.fill_diagonal(omega, 0.0)
    diag = vol - omega.sum(axis=1)
    if np.any(diag < 0):
        raise ValueError("intra/inter ratio infeasible for these block volumes")
    np.fill_diagonal(omega, diag)
    theta = tdeg / vol[block_of]                        # sums to 1 in each block
    src, dst = sample_edges(rng, theta, omega, sizes)
    perm = rng.permutation(n)                           # old id -> new id
    row_ptr, col_idx = edges_to_csr(n, perm[src], perm[dst])
    planted = np.empty(n, dtype=np.int32)
    planted[perm] = block_of
    info = {"n": n, "k": k, "alpha": alpha, "gamma": gamma, "d_min": d_min,
            "d_max": d_max, "rho": rho, "seed": seed,
            "nnz": int(row_ptr[-1]), "edges": int(row_ptr[-1]) // 2,
            "expected_mean_degree": float(tdeg.mean())}
    return Graph(n, row_ptr, col_idx, planted, info)


def two_cliques(m):
    """Two K_m cliques joined by one bridge edge (nodes 0..m-1, m..2m-1)."""
    src, dst = [], []
    for base in (0, m):
        for i in range(m):
            for j in range(i + 1, m):
                src.append(base + i)
                dst.append(base + j)
    src.append(m - 1)
    dst.append(m)
    rp, ci = edges_to_csr(2 * m, src, dst)
    planted = np.repeat(np.arange(2), m).astype(np.int32)
    return Graph(2 * m, rp, ci, planted, {"kind": "two_cliques", "m": m})


def clique_ring(c, m):
    """c cliques K_m in a ring, consecutive cliques joined by one edge."""
    src, dst = [], []
    for b in range(c):
        base = b * m
        for i in range(m):
            for j in range(i + 1, m):
                src.append(base + i)
                dst.append(base + j)
        src.append(base + m - 1)
        dst.append(((b + 1) % c) * m)
    rp, ci = edges_to_csr(c * m, src, dst)
    planted = np.repeat(np.arange(c), m).astype(np.int32)
    return Graph(c * m, rp, ci, planted, {"kind": "clique_ring", "c": c, "m": m})


def planted_small(n, k, p_in, p_out, seed):
    """Tiny Erdos-Renyi planted partition (for brute-force tests)."""
    rng = np.random.default_rng(np.random.SeedSequence([0x5C, int(seed)]))
    lab = np.arange(n) % k
    iu, ju = np.triu_indices(n, 1)
    p = np.where(lab[iu] == lab[ju], p_in, p_out)
    keep = rng.random(iu.size) < p
    rp, ci = edges_to_csr(n, iu[keep], ju[keep])
    return Graph(n, rp, ci, lab.astype(np.int32), {"kind": "planted_small"})


def bfs_ball(g, size, root=0):
    """Induced subgraph on the first `size` nodes reached by a breadth-first
    search from `root` (neighbours visited in column order), relabelled in
    visit order; degrees are those inside the subgraph.  If the component
    of `root` is smaller, the search restarts from the lowest unvisited
    node."""
    size = min(int(size), g.n)
    order = np.full(g.n, -1, dtype=np.int64)
    seq = []
    nxt = int(root)
    while len(seq) < size:
        while order[nxt] >= 0:
            nxt += 1
        order[nxt] = len(seq)
        seq.append(nxt)
        head = len(seq) - 1
        while head < len(seq) and len(seq) < size:
            u = seq[head]
            head += 1
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if order[v] < 0 and len(seq) < size:
                    order[v] = len(seq)
                    seq.append(int(v))
        nxt = 0
    nodes = np.asarray(seq, dtype=np.int64)
    src, dst = [], []
    for new_u, u in enumerate(nodes):
        nb = g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]
        nb_new = order[nb]
        keep = (nb_new >= 0) & (nb_new > new_u)
        src.append(np.full(int(keep.sum()), new_u))
        dst.append(nb_new[keep])
    rp, ci = edges_to_csr(size, np.concatenate(src), np.concatenate(dst))
    planted = g.planted[nodes].astype(np.int32) if g.planted.size else g.planted
    return Graph(size, rp, ci, planted, {"kind": "bfs_ball", "root": int(root),
                                          "parent": dict(g.info)})
