"""Pins of the projection operators (Sec. III-A) and the GCN (Sec. III-B)
against closed-form eigenpairs, invariants and dense NumPy matrices."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import gcn, graph, projection
from synth import dcsbm, two_cliques


def _dense(g):
    a = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[rows, g.col_idx] = 1.0
    return a


@pytest.fixture(scope="module")
def tiny():
    return dcsbm(48, 3, gamma=2.5, d_min=3, d_max=12, rho=3.0, seed=2, min_block=5)


def test_ncut_operator_eigenpair_and_radius(small_graph):
    g, _ = small_graph
    m = projection.ncut_operator(g.row_ptr, g.col_idx, g.n)
    d = graph.degrees(g.row_ptr).astype(float)
    assert d.min() > 0
    v = np.sqrt(d)
    np.testing.assert_allclose(m @ v, v, rtol=0, atol=1e-12 * v.max())
    lam = sla.eigsh(m, k=2, which="LM", return_eigenvectors=False)
    assert np.max(np.abs(lam)) <= 1.0 + 1e-12
    assert abs(np.max(lam) - 1.0) < 1e-10


def test_ncut_operator_dense(tiny):
    a = _dense(tiny)
    d = a.sum(1)
    s = np.where(d > 0, d ** -0.5, 0.0)
    ref = s[:, None] * a * s[None, :]
    m = projection.ncut_operator(tiny.row_ptr, tiny.col_idx, tiny.n).toarray()
    np.testing.assert_allclose(m, ref, rtol=1e-15, atol=0)


def test_modularity_operator_invariants(small_graph):
    g, _ = small_graph
    a = graph.adjacency(g.row_ptr, g.col_idx, g.n)
    d = graph.degrees(g.row_ptr).astype(float)
    m2 = float(graph.two_e(g.row_ptr))
    ones = np.ones((g.n, 1))
    b1 = projection.apply_modularity(a, d, m2, ones)
    assert np.max(np.abs(b1)) <= 1e-12 * d.max()          # B 1 = 0
    x = np.random.default_rng(0).standard_normal((g.n, 3))
    y = np.random.default_rng(1).standard_normal((g.n, 3))
    # symmetry: x^T B y == y^T B x
    lhs = x.T @ projection.apply_modularity(a, d, m2, y)
    rhs = (y.T @ projection.apply_modularity(a, d, m2, x)).T
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-9)


def test_modularity_operators_dense(tiny):
    a = _dense(tiny)
    d = a.sum(1)
    m2 = d.sum()
    q = a - np.outer(d, d) / m2                              # Eq. 4
    r = projection.theta(3, tiny.n, 8)
    got = projection.project(tiny.row_ptr, tiny.col_idx, tiny.n, projection.MOD_FULL, 8, 1, 3)
    np.testing.assert_allclose(got, q @ r, rtol=1e-12, atol=1e-12)
    qt = np.where(a > 0, q, 0.0)                             # reduced Q~ (Sec. III-A)
    got = projection.project(tiny.row_ptr, tiny.col_idx, tiny.n, projection.MOD_REDUCED, 8, 1, 3)
    np.testing.assert_allclose(got, qt @ r, rtol=1e-12, atol=1e-12)
    got = projection.project(tiny.row_ptr, tiny.col_idx, tiny.n, projection.MOD_FULL, 8, 3, 3)
    np.testing.assert_allclose(got, q @ q @ q @ r, rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("q", [1, 3])
def test_ncut_projection_dense(tiny, q):
    a = _dense(tiny)
    s = a.sum(1) ** -0.5
    m = s[:, None] * a * s[None, :]
    r = projection.theta(5, tiny.n, 12)
    got = projection.project(tiny.row_ptr, tiny.col_idx, tiny.n, projection.NCUT, 12, q, 5)
    np.testing.assert_allclose(got, np.linalg.matrix_power(m, q) @ r, rtol=1e-12, atol=1e-13)


def test_isolated_node_scale_is_zero():
    from synth.dcsbm import edges_to_csr
    rp, ci = edges_to_csr(4, [0, 1], [1, 2])                 # node 3 isolated
    m = projection.ncut_operator(rp, ci, 4).toarray()
    assert np.all(m[3] == 0) and np.all(np.isfinite(m))


def test_gcn_operator_eigenpair(small_graph):
    g, _ = small_graph
    ah = gcn.gcn_operator(g.row_ptr, g.col_idx, g.n)
    v = np.sqrt(graph.degrees(g.row_ptr) + 1.0)
    np.testing.assert_allclose(ah @ v, v, rtol=1e-13)
    lam = sla.eigsh(ah, k=1, which="LA", return_eigenvectors=False)
    assert abs(lam[0] - 1.0) < 1e-10


def test_gcn_dense_eq6(tiny):
    a = _dense(tiny) + np.eye(tiny.n)
    dh = a.sum(1) ** -0.5
    an = dh[:, None] * a * dh[None, :]
    y = projection.project(tiny.row_ptr, tiny.col_idx, tiny.n, projection.NCUT, 16, 2, 9)
    h = y
    dims = [12, 8]
    l_in = 16
    for k, l_out in enumerate(dims, 1):
        w = gcn.weight(9, k, l_in, l_out)
        z = np.tanh(an @ h @ w)
        h = z / np.linalg.norm(z, axis=1, keepdims=True)
        l_in = l_out
    got = gcn.embed(tiny.row_ptr, tiny.col_idx, tiny.n, y, dims, 9)
    np.testing.assert_allclose(got, h, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(got, axis=1), 1.0, rtol=1e-14)


def test_gcn_weight_scale():
    w = gcn.weight(0, 1, 256, 64)
    assert abs(w.std() - 256 ** -0.5) < 0.05 * 256 ** -0.5
    assert not np.array_equal(w[:64], gcn.weight(0, 2, 256, 64)[:64])


def test_two_cliques_embedding_separates():
    g = two_cliques(5)
    y = projection.project(g.row_ptr, g.col_idx, g.n, projection.MOD_FULL, 64, 1, 0)
    z = gcn.embed(g.row_ptr, g.col_idx, g.n, y, [64, 64], 0)
    # within-clique distances are smaller than across
    d = ((z[:, None, :] - z[None, :, :]) ** 2).sum(-1)
    same = g.planted[:, None] == g.planted[None, :]
    assert d[same].max() < d[~same].min()


def test_row_normalize_zero_row_floor():
    """Sec. III-B normalises rows; a zero row (an isolated node under NCut,
    whose row of M is zero) is divided by the floor 1e-12 and stays zero,
    and a row below the floor is divided by the floor, not by its norm."""
    z = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [1e-13, 0.0, 0.0]])
    got = gcn.row_normalize(z)
    assert np.array_equal(got[0], np.zeros(3))
    assert np.array_equal(got[1], np.array([0.6, 0.8, 0.0]))
    np.testing.assert_allclose(got[2], [0.1, 0.0, 0.0], rtol=1e-15, atol=0)


def _graph_with_isolated():
    from synth.dcsbm import edges_to_csr
    # a path 0-1-2-3, a triangle 4-5-6, node 7 isolated, a star 8-{9,10,11}
    return edges_to_csr(12, [0, 1, 2, 4, 5, 4, 8, 8, 8], [1, 2, 3, 5, 6, 6, 9, 10, 11])


@pytest.mark.parametrize("normalize_input", [False, True])
def test_gcn_dense_eq6_isolated_node_and_input_normalisation(normalize_input):
    """Dense Eq. 6 on a graph with an isolated node, with and without the
    row normalisation of Y before the first layer: the isolated node's Y row
    is zero under NCut (D^-1/2 = 0), its row of A_hat_n is e_i, so its
    embedding row stays zero through every layer."""
    rp, ci = _graph_with_isolated()
    n = 12
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    a[rows, ci] = 1.0
    y = projection.project(rp, ci, n, projection.NCUT, 16, 2, 4)
    assert np.all(y[7] == 0) and np.all(y[np.arange(n) != 7].any(axis=1))
    ah = a + np.eye(n)
    dh = ah.sum(1) ** -0.5
    an = dh[:, None] * ah * dh[None, :]
    h = y.copy()
    if normalize_input:
        nrm = np.sqrt((h * h).sum(1))
        h = h / np.where(nrm > 1e-12, nrm, 1e-12)[:, None]
        assert np.all(h[7] == 0)
    l_in = 16
    for k, l_out in enumerate([12, 8], 1):
        w = gcn.weight(4, k, l_in, l_out)
        z = np.tanh(an @ h @ w)
        nrm = np.sqrt((z * z).sum(1))
        h = z / np.where(nrm > 1e-12, nrm, 1e-12)[:, None]
        l_in = l_out
    got = gcn.embed(rp, ci, n, y, [12, 8], 4, normalize_input=normalize_input)
    np.testing.assert_allclose(got, h, rtol=1e-12, atol=1e-14)
    assert np.all(got[7] == 0)
    other = gcn.embed(rp, ci, n, y, [12, 8], 4, normalize_input=not normalize_input)
    assert np.abs(got - other).max() > 1e-3          # the flag changes the embedding
