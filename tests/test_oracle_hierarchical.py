"""Pins of the hierarchical model selection (Sec. III-C, Alg. 1) and local
modularity (Eq. 7): LMod over U = V is Eq. 3 modularity (networkx), LMod
against its double-sum form on random subsets, closed forms on cliques joined
by bridges, each branch of the stopping rule, brute force of the root decision
on small graphs, and planted cliques recovered end to end."""
import itertools

import networkx as nx
import numpy as np
import pytest

from oracle import hierarchical as hier
from oracle import pipeline, projection, scores
from synth import clique_ring, dcsbm, planted_small, two_cliques


def _nxg(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col_idx.tolist()))
    return G


def _lmod_double_sum(g, part):
    """(1 / 2e_U) sum_{i,j in U} [A_ij - d_i d_j / 2e_U] [c_i = c_j] with d the
    degrees in G: the pairwise form of Eq. 7 (sum over ordered pairs of a
    block of A_ij is 2 m_r, of d_i d_j is vol_r^2)."""
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col_idx] = 1.0
    d = A.sum(1)
    u = np.flatnonzero(part >= 0)
    two_e = d[u].sum()
    total = 0.0
    for i in u:
        for j in u:
            if part[i] == part[j]:
                total += A[i, j] - d[i] * d[j] / two_e
    return total / two_e


def test_lmod_over_all_nodes_is_modularity():
    g = dcsbm(400, 5, gamma=2.5, d_min=4, d_max=40, rho=3.0, seed=3)
    G = _nxg(g)
    rng = np.random.default_rng(0)
    for k in (1, 2, 5, 9):
        lab = rng.integers(0, k, g.n)
        comms = [set(np.flatnonzero(lab == r).tolist()) for r in range(k)]
        comms = [c for c in comms if c]
        ref = nx.algorithms.community.modularity(G, comms)
        got = hier.lmod(g.row_ptr, g.col_idx, lab, k)
        assert abs(got - ref) < 1e-12
        assert abs(got - scores.modularity(g.row_ptr, g.col_idx, lab)) < 1e-12


def test_lmod_double_sum_on_subsets():
    g = planted_small(24, 3, 0.7, 0.15, seed=4)
    rng = np.random.default_rng(1)
    for trial in range(20):
        part = np.full(g.n, -1)
        u = rng.choice(g.n, size=rng.integers(3, g.n), replace=False)
        k = int(rng.integers(1, 4))
        part[u] = rng.integers(0, k, u.size)
        got = hier.lmod(g.row_ptr, g.col_idx, part, k)
        if got is None:
            continue
        assert abs(got - _lmod_double_sum(g, part)) < 1e-12, trial


def test_lmod_counts_degrees_outside_the_subset():
    """Two K6 joined by a bridge, U = one clique (nodes 0..5): its degrees in G
    sum to 31 (the bridge end has degree 6), m_U = 15, so LMod(U) as a single
    block is 15 / 15.5 - 1 = -1/31, while the modularity of G[U] would be 0."""
    g = two_cliques(6)
    part = np.full(g.n, -1)
    part[:6] = 0
    m, vol = hier.lmod_counts(g.row_ptr, g.col_idx, part, 1)
    assert m.tolist() == [15] and vol.tolist() == [31]
    assert abs(hier.lmod(g.row_ptr, g.col_idx, part, 1) - (-1.0 / 31.0)) < 1e-15
    # the two cliques over U = V: 2 (15/31) - 2 (31/62)^2 = 30/31 - 1/2
    lab = np.repeat([0, 1], 6)
    assert abs(hier.lmod(g.row_ptr, g.col_idx, lab, 2) - (30 / 31 - 0.5)) < 1e-15


def _one_hot_splitter(truth):
    """Splits U by the planted label: the lowest planted label present in U
    against the rest (a stand-in for KMeans with a perfect embedding)."""
    def split(nodes, depth):
        lab = truth[nodes]
        return (lab != lab.min()).astype(np.int64)
    return split


def test_two_cliques_split_once():
    """Root (12 nodes > 2 eps + 1): m_1 = 0, m_2 = 30/31 - 1/2 > m_1 and both
    sides have 6 > eps nodes, so it splits; each clique has 6 <= 11 nodes and
    becomes a block."""
    g = two_cliques(6)
    out = hier.partition(g.row_ptr, g.col_idx, None, splitter=_one_hot_splitter(g.planted))
    assert out["labels"].tolist() == [0] * 6 + [1] * 6
    root = out["tree"][0]
    assert root[2] == "split" and abs(root[3]) < 1e-15
    assert abs(root[4] - (30 / 31 - 0.5)) < 1e-15


def test_stopping_rule_small_side():
    """A side with <= eps nodes stops the recursion even when m_2 > m_1."""
    g = two_cliques(6)

    def lopsided(nodes, depth):
        s = np.zeros(nodes.size, dtype=np.int64)
        s[:5] = 1                              # |U_2| = 5 = eps
        return s
    out = hier.partition(g.row_ptr, g.col_idx, None, splitter=lopsided)
    assert out["k"] == 1 and out["tree"][0][2] == "block"
    # and the same sides swapped (|U_1| = 5)
    out = hier.partition(g.row_ptr, g.col_idx, None,
                         splitter=lambda nodes, depth: 1 - lopsided(nodes, depth))
    assert out["k"] == 1


def test_stopping_rule_modularity_drop():
    """K12: every split lowers LMod (m_1 = 0 > m_2), so the clique stays one
    block; for the 6 + 6 split m_2 = 30/66 - 1/2 exactly."""
    src, dst = np.triu_indices(12, 1)
    from synth.dcsbm import edges_to_csr
    rp, ci = edges_to_csr(12, src, dst)
    out = hier.partition(rp, ci, None,
                         splitter=lambda nodes, depth: (nodes >= 6).astype(np.int64))
    assert out["k"] == 1
    root = out["tree"][0]
    assert root[2] == "block" and abs(root[4] - (30 / 66 - 0.5)) < 1e-15


def test_small_sets_are_blocks_without_kmeans():
    g = two_cliques(5)                          # 10 nodes <= 2 eps + 1

    def never(nodes, depth):
        raise AssertionError("KMeans must not run on a set of <= 2 eps + 1 nodes")
    out = hier.partition(g.row_ptr, g.col_idx, None, splitter=never)
    assert out["k"] == 1


def test_root_decision_brute_force():
    """On small graphs, the root decision for every 2-split of V with both
    sides > eps is: split iff the two-block modularity (brute-force pair sum)
    is >= that of V as one block (0)."""
    g = planted_small(12, 2, 0.9, 0.1, seed=7)
    for mask in itertools.islice(itertools.product([0, 1], repeat=11), 0, 2048, 7):
        side = np.array((0,) + mask, dtype=np.int64)
        if min(np.sum(side == 0), np.sum(side == 1)) <= hier.EPS:
            continue
        out = hier.partition(g.row_ptr, g.col_idx, None,
                             splitter=lambda nodes, depth, s=side: s[nodes])
        m2 = _lmod_double_sum(g, side)
        root = out["tree"][0]
        assert abs(root[4] - m2) < 1e-12
        assert root[2] == ("block" if 0.0 > m2 else "split")


def test_ring_of_cliques_with_given_splits():
    g = clique_ring(4, 8)
    out = hier.partition(g.row_ptr, g.col_idx, None, splitter=_one_hot_splitter(g.planted))
    assert out["k"] == 4
    assert scores.nmi(out["labels"], g.planted) == 1.0
    # depth-first numbering: block r is clique r (U_1 = the lowest planted label)
    assert out["labels"].tolist() == g.planted.tolist()


@pytest.mark.parametrize("op", [projection.NCUT, projection.MOD_FULL])
def test_embedding_recovers_planted_cliques(op):
    """The whole path (projection, GCN, Alg. 1 with KMeans) on a ring of six
    K12 cliques recovers the cliques."""
    g = clique_ring(6, 12)
    cfg = pipeline.Config(op=op, proj_dim=32, q=3, layer_dims=[32, 32])
    y = projection.project(g.row_ptr, g.col_idx, g.n, op, cfg.proj_dim, cfg.q, 0)
    from oracle import gcn
    z = gcn.embed(g.row_ptr, g.col_idx, g.n, y, cfg.layer_dims, 0)
    out = hier.partition(g.row_ptr, g.col_idx, z, seed=0)
    assert out["k"] == 6
    assert scores.nmi(out["labels"], g.planted) == 1.0


def test_race_draws_depend_on_depth_not_order():
    nodes = np.array([3, 10, 42, 77], dtype=np.int64)
    e0 = hier.race_exponentials(0, nodes, 0, 0)
    e1 = hier.race_exponentials(0, nodes, 0, 1)
    assert not np.any(e0 == e1)
    sub = hier.race_exponentials(0, nodes[2:], 0, 0)
    assert np.array_equal(sub, e0[2:])
