"""Partition scores, model selection and NMI (oracle side).

Modularity, Eq. 3: Mod = (1/2e) sum_r sum_{i,j in C_r} [A_ij - d_i d_j / 2e].
Summing over ordered pairs, sum_{i,j in C_r} A_ij = 2 l_r (l_r = intra-block
edges) and sum_{i,j in C_r} d_i d_j = vol_r^2, so
    Mod = sum_r ( l_r / e - (vol_r / 2e)^2 ).
NCut, Eq. 1: NCut = 1/2 sum_r cut(C_r, rest) / vol(C_r), cut_r = vol_r - 2 l_r;
blocks with vol_r = 0 contribute nothing.

The integer counts l_r, vol_r are exact; the FP64 finish runs over r in
ascending order (term by term, left to right) so any implementation that uses
the same counts and the same operation order gets the same bits.

Model selection over the candidate grid: K* is the first candidate (in grid
order) whose modularity equals the maximum; the selected labels are relabelled
by first occurrence in node order.

NMI = 2 I(a;b) / (H(a) + H(b)) in natural log (arithmetic normalisation); 1 if
both labelings are constant.

Pinned in ``tests/test_oracle_scores.py``: closed forms on two cliques joined
by a bridge, networkx modularity, the dense double sum of Eq. 3, brute force
over all set partitions of tiny graphs, and scikit-learn's NMI.
"""
import numpy as np


def block_counts(row_ptr, col_idx, labels, k):
    """(l_r, vol_r) int64 arrays of length k for one labeling."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    n = row_ptr.size - 1
    deg = np.diff(row_ptr)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    same = labels[rows] == labels[col_idx]
    twice_l = np.bincount(labels[rows[same]], minlength=k).astype(np.int64)
    vol = np.bincount(labels, weights=deg, minlength=k).astype(np.int64)
    assert np.all(twice_l % 2 == 0)
    return twice_l // 2, vol


def modularity_from_counts(l, vol, m2):
    e = float(m2 // 2)
    m2f = float(m2)
    total = 0.0
    for r in range(len(l)):
        t = float(vol[r]) / m2f
        total = total + (float(l[r]) / e - t * t)
    return total


def ncut_from_counts(l, vol):
    total = 0.0
    for r in range(len(l)):
        if vol[r] > 0:
            total = total + float(vol[r] - 2 * l[r]) / float(vol[r])
    return 0.5 * total


def modularity(row_ptr, col_idx, labels, k=None):
    labels = np.asarray(labels, dtype=np.int64)
    k = int(labels.max()) + 1 if k is None else k
    l, vol = block_counts(row_ptr, col_idx, labels, k)
    return modularity_from_counts(l, vol, int(np.asarray(row_ptr)[-1]))


def ncut(row_ptr, col_idx, labels, k=None):
    labels = np.asarray(labels, dtype=np.int64)
    k = int(labels.max()) + 1 if k is None else k
    l, vol = block_counts(row_ptr, col_idx, labels, k)
    return ncut_from_counts(l, vol)


def score_candidates(row_ptr, col_idx, labels_all, ks):
    """Mod and NCut per candidate column of labels_all [n, len(ks)]."""
    m2 = int(np.asarray(row_ptr)[-1])
    mod = np.zeros(len(ks))
    nc = np.zeros(len(ks))
    for j, k in enumerate(ks):
        l, vol = block_counts(row_ptr, col_idx, labels_all[:, j], k)
        mod[j] = modularity_from_counts(l, vol, m2)
        nc[j] = ncut_from_counts(l, vol)
    return mod, nc


def canonical(labels):
    """Relabel by first occurrence in node order; returns (labels, K_eff)."""
    labels = np.asarray(labels, dtype=np.int64)
    _, first = np.unique(labels, return_index=True)
    order = np.argsort(first, kind="stable")
    uniq = np.unique(labels)[order]
    remap = np.empty(int(labels.max()) + 1, dtype=np.int64)
    remap[uniq] = np.arange(uniq.size)
    return remap[labels], int(uniq.size)


def select(mod):
    """Index of the first maximum of mod (exact FP64 comparison)."""
    mod = np.asarray(mod, dtype=np.float64)
    best = 0
    for j in range(1, mod.size):
        if mod[j] > mod[best]:
            best = j
    return best


def entropy(labels):
    _, cnt = np.unique(labels, return_counts=True)
    p = cnt / cnt.sum()
    return float(-np.sum(p * np.log(p)))


def nmi(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    ha, hb = entropy(a), entropy(b)
    if ha + hb == 0.0:
        return 1.0
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    n = a.size
    joint = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(joint, (ai, bi), 1.0)
    pj = joint / n
    pa = pj.sum(axis=1, keepdims=True)
    pb = pj.sum(axis=0, keepdims=True)
    nz = pj > 0
    mi = float(np.sum(pj[nz] * np.log(pj[nz] / (pa @ pb)[nz])))
    return 2.0 * mi / (ha + hb)
