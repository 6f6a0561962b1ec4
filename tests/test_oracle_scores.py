"""Pins of modularity (Eq. 3), NCut (Eq. 1), selection and NMI: closed forms,
networkx, the dense double sum of Eq. 3, brute force over all set partitions
of tiny graphs, and scikit-learn's NMI."""
import json
import os

import networkx as nx
import numpy as np
import pytest

from oracle import pipeline, projection, scores
from synth import clique_ring, dcsbm, planted_small, two_cliques

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _nxg(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col_idx.tolist()))
    return G


def test_two_cliques_closed_form():
    with open(os.path.join(GOLDEN, "two_cliques_closed_form.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        g = two_cliques(c["m"])
        mod = scores.modularity(g.row_ptr, g.col_idx, g.planted)
        nc = scores.ncut(g.row_ptr, g.col_idx, g.planted)
        assert abs(mod - c["mod_num"] / c["mod_den"]) < 1e-15
        assert abs(nc - c["ncut_num"] / c["ncut_den"]) < 1e-15


def test_degenerate_partitions(small_graph):
    g, _ = small_graph
    one = np.zeros(g.n, dtype=np.int64)
    assert abs(scores.modularity(g.row_ptr, g.col_idx, one)) < 1e-15
    assert scores.ncut(g.row_ptr, g.col_idx, one) == 0.0
    single = np.arange(g.n)
    d = np.diff(g.row_ptr).astype(float)
    m2 = d.sum()
    assert abs(scores.modularity(g.row_ptr, g.col_idx, single) + np.sum((d / m2) ** 2)) < 1e-14
    # every singleton block is fully cut: NCut = n/2 for no isolated nodes
    assert abs(scores.ncut(g.row_ptr, g.col_idx, single) - g.n / 2) < 1e-9


def test_modularity_matches_networkx_and_dense(small_graph):
    g, _ = small_graph
    G = _nxg(g)
    rng = np.random.default_rng(0)
    a = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[rows, g.col_idx] = 1
    d = a.sum(1)
    m2 = d.sum()
    for labels in (g.planted, rng.integers(0, 7, g.n)):
        comms = [set(np.flatnonzero(labels == r).tolist()) for r in np.unique(labels)]
        ref = nx.algorithms.community.modularity(G, comms)
        got = scores.modularity(g.row_ptr, g.col_idx, labels)
        assert abs(got - ref) < 1e-12
        same = labels[:, None] == labels[None, :]
        dense = np.sum((a - np.outer(d, d) / m2) * same) / m2      # Eq. 3 double sum
        assert abs(got - dense) < 1e-12
        # NCut from its definition: cut(C_r, rest) / vol(C_r), Eq. 1
        nc = 0.0
        for r in np.unique(labels):
            inr = labels == r
            nc += a[np.ix_(inr, ~inr)].sum() / d[inr].sum()
        assert abs(scores.ncut(g.row_ptr, g.col_idx, labels) - 0.5 * nc) < 1e-12


def _set_partitions(n):
    """All restricted growth strings of length n (every set partition once)."""
    parts = [[0]]
    for _ in range(1, n):
        nxt = []
        for p in parts:
            m = max(p)
            for v in range(m + 2):
                nxt.append(p + [v])
        parts = nxt
    return np.array(parts, dtype=np.int8)


def _brute_force_best(g):
    a = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[rows, g.col_idx] = 1
    d = a.sum(1)
    m2 = d.sum()
    q = (a - np.outer(d, d) / m2) / m2
    parts = _set_partitions(g.n)
    best_val, best = -np.inf, None
    for chunk in np.array_split(parts, max(1, len(parts) // 20000)):
        same = chunk[:, :, None] == chunk[:, None, :]
        vals = np.einsum("bij,ij->b", same, q)
        i = int(np.argmax(vals))
        if vals[i] > best_val:
            best_val, best = vals[i], chunk[i]
    return best_val, best


def _same_partition(a, b):
    return scores.nmi(a, b) > 1 - 1e-12


@pytest.mark.parametrize("maker", [lambda: two_cliques(5), lambda: clique_ring(3, 3)])
def test_pipeline_reaches_brute_force_optimum(maker):
    g = maker()
    best_val, best = _brute_force_best(g)
    for op in (projection.NCUT, projection.MOD_FULL, projection.MOD_REDUCED):
        cfg = pipeline.Config(op=op, proj_dim=64, q=1, layer_dims=[64, 64],
                              k_min=2, k_max=5, seed=0)
        r = pipeline.run(g.row_ptr, g.col_idx, g.n, cfg)
        assert r["mod"][r["best"]] <= best_val + 1e-12
        assert abs(r["mod"][r["best"]] - best_val) < 1e-12
        assert _same_partition(r["labels"], best)
        assert r["k_star"] == len(set(best.tolist()))


def test_brute_force_bounds_random_graphs():
    for s in range(3):
        g = planted_small(9, 3, 0.8, 0.15, s)
        if g.nnz == 0:
            continue
        best_val, _ = _brute_force_best(g)
        cfg = pipeline.Config(op=projection.NCUT, proj_dim=32, q=2, layer_dims=[32, 16],
                              k_min=1, k_max=6, seed=s)
        r = pipeline.run(g.row_ptr, g.col_idx, g.n, cfg)
        assert np.all(r["mod"] <= best_val + 1e-12)


def test_selection_first_max_and_canonical():
    assert scores.select([0.1, 0.3, 0.3, 0.2]) == 1
    lab, k = scores.canonical(np.array([5, 5, 2, 9, 2]))
    assert lab.tolist() == [0, 0, 1, 2, 1] and k == 3


def test_nmi_matches_sklearn():
    from sklearn.metrics import normalized_mutual_info_score as sk
    rng = np.random.default_rng(0)
    for _ in range(5):
        a = rng.integers(0, 6, 500)
        b = rng.integers(0, 4, 500)
        assert abs(scores.nmi(a, b) - sk(a, b)) < 1e-12
    a = rng.integers(0, 6, 500)
    assert abs(scores.nmi(a, (a + 3) % 6) - 1.0) < 1e-12
    assert scores.nmi(np.zeros(10), np.zeros(10)) == 1.0
