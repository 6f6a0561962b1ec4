"""Pins of CSR validation, degrees and 2e against networkx / scipy."""
import networkx as nx
import numpy as np
import pytest

from oracle import graph
from synth import dcsbm, two_cliques
from synth.dcsbm import edges_to_csr


def _nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col_idx.tolist()))
    return G


def test_degrees_and_edges_match_networkx(small_graph):
    g, _ = small_graph
    G = _nx(g)
    deg = graph.degrees(g.row_ptr)
    assert np.array_equal(deg, np.array([G.degree(i) for i in range(g.n)]))
    assert graph.two_e(g.row_ptr) == 2 * G.number_of_edges()
    graph.validate_csr(g.row_ptr, g.col_idx, g.n)


def _bad(rp, ci, n):
    with pytest.raises(graph.CSRError):
        graph.validate_csr(np.array(rp), np.array(ci), n)


def test_rejects_malformed():
    g = two_cliques(4)
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    graph.validate_csr(rp, ci, g.n)
    _bad(rp[:-1], ci, g.n)                       # wrong length
    c2 = ci.copy(); c2[0] = 9; _bad(rp, c2, g.n)  # out of range
    c3 = ci.copy(); c3[0], c3[1] = c3[1], c3[0]; _bad(rp, c3, g.n)   # unsorted
    c4 = ci.copy(); c4[1] = c4[0]; _bad(rp, c4, g.n)                  # duplicate
    c5 = ci.copy(); c5[0] = 0; _bad(rp, c5, g.n)                      # self loop
    # asymmetric: drop one direction of an edge
    rp6, ci6 = edges_to_csr(3, [0, 1], [1, 2])
    ci6 = ci6.copy(); ci6[-1] = 0                                     # row 2: 1 -> 0
    _bad(rp6, ci6, 3)
    rp7 = rp.copy(); rp7[0] = 1; _bad(rp7, ci, g.n)


def test_generator_statistics():
    # expected intra/inter ratio and mean degree close to the recipe
    g = dcsbm(4000, 8, gamma=2.5, d_min=10, d_max=100, rho=2.5, seed=3)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    same = g.planted[rows] == g.planted[g.col_idx]
    ratio = same.sum() / (~same).sum()
    assert abs(ratio - 2.5) < 0.25
    mean_deg = g.nnz / g.n
    assert abs(mean_deg - g.info["expected_mean_degree"]) < 0.1 * g.info["expected_mean_degree"]
    assert np.bincount(g.planted).min() >= 10
    graph.validate_csr(g.row_ptr, g.col_idx, g.n)


def test_generator_expected_edge_count_closed_form():
    """E|E| = sum over node pairs of P(Pois(lambda_ij) >= 1) = 1 - exp(-lambda_ij)
    for fixed theta and Omega (SBM definition, Sec. II)."""
    from synth.dcsbm import sample_edges
    rng = np.random.default_rng(7)
    sizes = np.array([20, 30, 25])
    k = sizes.size
    block_of = np.repeat(np.arange(k), sizes)
    raw = rng.uniform(1, 5, sizes.sum())
    theta = raw / np.bincount(block_of, weights=raw)[block_of]
    omega = np.array([[60.0, 8, 5], [8, 90, 10], [5, 10, 70]])
    n = sizes.sum()
    lam = theta[:, None] * theta[None, :] * omega[block_of][:, block_of]
    iu, ju = np.triu_indices(n, 1)
    expect = np.sum(1.0 - np.exp(-lam[iu, ju]))
    var = np.sum(np.exp(-lam[iu, ju]) * (1.0 - np.exp(-lam[iu, ju])))
    reps = 400
    tot = 0
    pair_hits = np.zeros((k, k))
    for _ in range(reps):
        src, dst = sample_edges(rng, theta, omega, sizes)
        rp, ci = edges_to_csr(n, src, dst)
        tot += rp[-1] // 2
        rows = np.repeat(np.arange(n), np.diff(rp))
        np.add.at(pair_hits, (block_of[rows], block_of[ci]), 1)
    mean = tot / reps
    assert abs(mean - expect) < 4 * np.sqrt(var / reps)
    # per block pair: expected edge-end counts
    exp_pair = np.zeros((k, k))
    p1 = 1.0 - np.exp(-lam)
    np.fill_diagonal(p1, 0.0)
    for r in range(k):
        for s in range(k):
            exp_pair[r, s] = p1[np.ix_(block_of == r, block_of == s)].sum()
    np.testing.assert_allclose(pair_hits / reps, exp_pair, rtol=0.05)
