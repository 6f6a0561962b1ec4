"""Hierarchical model selection with local modularity (oracle side).

Sec. III-C, Alg. 1 (hierarchical model selection) and Eq. 7 (local
modularity).  For a node set U of G split into blocks U_1..U_K:

    LMod(U_1..U_K; G) = sum_r [ m_r / e_U - (vol_r / 2 e_U)^2 ]

with m_r the number of edges of G with both ends in U_r, vol_r the sum of the
degrees in G (not in G[U]) of the nodes of U_r, and 2 e_U = sum_r vol_r, the
total G-degree of U.  With U = V this is the modularity of Eq. 3.

Alg. 1 partitions U recursively: m_1 = LMod(U; G) (U as one block), KMeans
with K = 2 on the embeddings of U gives (U_1, U_2), m_2 = LMod(U_1, U_2; G);
U becomes a block when |U_1| <= eps or |U_2| <= eps or m_1 > m_2 (eps = 5),
otherwise U_1 and then U_2 are partitioned the same way.

Readings (the paper does not fix these):
* the printed stopping rule tests |U_1| twice; the text tests both sides, so
  |U_2| <= eps is the second test;
* KMeans with K = 2 is the flat grid's: k-means++ seeding by the exponential
  race and Lloyd to a fixed point or T_max, ties to the lower index, an empty
  cluster keeps its centre.  The race over U draws
  E_{t,i} = -ln u(Philox4x64-10, key (seed, 0x21), counter (i, t, depth, 0))
  with i the node's id in G and depth the level of U in the tree (the root
  is level 0): a node belongs to one set per level, so its draws never
  repeat, and they do not depend on the order the sets are processed in;
* U_1 is the cluster of the first pick;
* |U| <= 2 eps + 1: any split leaves one side with at most eps nodes, so U is
  a block without running KMeans (the outcome Alg. 1 reaches anyway);
* vol(U) = 0: e_U = 0 and LMod is undefined; U is a block;
* blocks are numbered in the order Alg. 1 adds them to C (depth first, U_1
  before U_2).

Pinned in ``tests/test_oracle_hierarchical.py``: LMod(V; C) equals Eq. 3
modularity, LMod equals its double-sum form on random subsets, closed forms
on cliques joined by bridges, the stopping rule case by case, brute force of
the root decision on small graphs, and planted blocks recovered on cliques.
"""
import numpy as np

from . import fmath, kmeans, philox

EPS = 5
STREAM_HIER_RACE = 0x21


def lmod_counts(row_ptr, col_idx, part, k):
    """(m_r, vol_r) int64 [k] for a labelling `part` over all N nodes in which
    nodes outside U carry -1 and nodes of U_r carry r."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    n = row_ptr.size - 1
    deg = np.diff(row_ptr)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    inside = part >= 0
    same = inside[rows] & (part[rows] == part[col_idx])
    twice_m = np.bincount(part[rows[same]], minlength=k).astype(np.int64)
    vol = np.bincount(part[inside], weights=deg[inside], minlength=k).astype(np.int64)
    assert np.all(twice_m % 2 == 0)
    return twice_m // 2, vol


def lmod_from_counts(m, vol):
    """Eq. 7 in FP64 from integer counts, r ascending, left to right."""
    two_e = int(np.sum(vol))
    e = two_e / 2.0
    total = 0.0
    for r in range(len(m)):
        t = float(vol[r]) / float(two_e)
        total = total + (float(m[r]) / e - t * t)
    return total


def lmod(row_ptr, col_idx, part, k):
    """LMod(U_1..U_k; G), Eq. 7 (None when vol(U) = 0)."""
    m, vol = lmod_counts(row_ptr, col_idx, part, k)
    if int(np.sum(vol)) == 0:
        return None
    return lmod_from_counts(m, vol)


def race_exponentials(seed, nodes, t, depth):
    """E_{t,i} = -ln u for the nodes of U (global ids), at tree level depth."""
    ctr = np.zeros((nodes.size, 4), dtype=np.uint64)
    ctr[:, 0] = nodes.astype(np.uint64)
    ctr[:, 1] = np.uint64(t)
    ctr[:, 2] = np.uint64(depth)
    blk = philox.philox4x64(ctr, np.array([seed, STREAM_HIER_RACE], dtype=np.uint64))
    return -fmath.ln(fmath.uniform52(blk[:, 0]))


def seed_two(z_u, nodes, seed, depth):
    """The first two k-means++ picks over U by the exponential race (positions
    into U; ties to the lower position, i.e. the lower node id)."""
    n = nodes.size
    picks = []
    w = np.ones(n, dtype=np.float64)
    picked = np.zeros(n, dtype=bool)
    for t in range(2):
        e = race_exponentials(seed, nodes, t, depth)
        pos = w > 0
        if np.any(pos):
            ratio = np.full(n, np.inf)
            ratio[pos] = e[pos] / w[pos]
            p = int(np.argmin(ratio))
        else:
            p = int(np.flatnonzero(~picked)[0])
        picks.append(p)
        picked[p] = True
        diff = z_u - z_u[p]
        w = np.sum(diff * diff, axis=1)
    return np.array(picks, dtype=np.int64)


def split_two(z, nodes, seed, depth, t_max=100):
    """KMeans with K = 2 on the embeddings of U: labels (0 = U_1, 1 = U_2) in
    the order of `nodes`."""
    z_u = np.asarray(z, dtype=np.float64)[nodes]
    picks = seed_two(z_u, nodes, seed, depth)
    lab, _, _ = kmeans.lloyd(z_u, z_u[picks], t_max)
    return lab


def partition(row_ptr, col_idx, z, seed=0, eps=EPS, t_max=100, splitter=None):
    """Alg. 1 from U = V.  Returns dict(labels [N] int64 (block number in the
    order blocks are added), tree (list of visited sets in depth-first order:
    (depth, nodes, decision, m1, m2, sizes))).

    `splitter(nodes, depth) -> labels` replaces the KMeans step when given
    (used to check the tree logic against given K = 2 labels)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.size - 1
    labels = np.full(n, -1, dtype=np.int64)
    tree = []
    nblocks = 0
    stack = [(np.arange(n, dtype=np.int64), 0)]
    while stack:
        nodes, depth = stack.pop()
        part = np.full(n, -1, dtype=np.int64)
        part[nodes] = 0
        m1 = lmod(row_ptr, col_idx, part, 1)
        if nodes.size <= 2 * eps + 1 or m1 is None:
            labels[nodes] = nblocks
            nblocks += 1
            tree.append((depth, nodes, "block", m1, None, None))
            continue
        side = splitter(nodes, depth) if splitter else split_two(z, nodes, seed, depth, t_max)
        u1, u2 = nodes[side == 0], nodes[side == 1]
        part[u2] = 1
        m2 = lmod(row_ptr, col_idx, part, 2)
        if u1.size <= eps or u2.size <= eps or m1 > m2:
            labels[nodes] = nblocks
            nblocks += 1
            tree.append((depth, nodes, "block", m1, m2, (u1.size, u2.size)))
            continue
        tree.append((depth, nodes, "split", m1, m2, (u1.size, u2.size)))
        stack.append((u2, depth + 1))     # U_1 is partitioned first
        stack.append((u1, depth + 1))
    return {"labels": labels, "k": nblocks, "tree": tree}
