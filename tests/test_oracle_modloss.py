"""Pins of the relaxed-modularity loss and the GCN adjoint: central finite
differences in FP64 and the closed form loss(one-hot S) = -Mod (Eq. 3)."""
import numpy as np
import pytest

from oracle import gcn, modloss, projection, scores
from synth import dcsbm, two_cliques


@pytest.fixture(scope="module")
def g():
    return dcsbm(120, 4, gamma=2.5, d_min=3, d_max=15, rho=3.0, seed=5, min_block=10)


def test_onehot_loss_is_minus_modularity(g):
    rng = np.random.default_rng(0)
    for k in (2, 4, 7):
        lab = rng.integers(0, k, g.n)
        s = np.eye(k)[lab]
        assert abs(modloss.loss_of_s(g.row_ptr, g.col_idx, g.n, s)
                   + scores.modularity(g.row_ptr, g.col_idx, lab, k)) < 1e-13
    c = two_cliques(5)
    s = np.eye(2)[c.planted]
    assert abs(modloss.loss_of_s(c.row_ptr, c.col_idx, c.n, s) + 19 / 42) < 1e-15


def test_grad_s_against_dense_and_fd(g):
    rng = np.random.default_rng(1)
    s = rng.random((g.n, 5))
    a = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[rows, g.col_idx] = 1
    d = a.sum(1)
    m2 = d.sum()
    bmat = a - np.outer(d, d) / m2
    np.testing.assert_allclose(modloss.grad_s(g.row_ptr, g.col_idx, g.n, s),
                               -2 * bmat @ s / m2, rtol=1e-12, atol=1e-14)
    h = 1e-6
    for (i, j) in [(0, 0), (7, 3), (50, 4)]:
        sp, sm = s.copy(), s.copy()
        sp[i, j] += h
        sm[i, j] -= h
        fd = (modloss.loss_of_s(g.row_ptr, g.col_idx, g.n, sp)
              - modloss.loss_of_s(g.row_ptr, g.col_idx, g.n, sm)) / (2 * h)
        assert abs(fd - modloss.grad_s(g.row_ptr, g.col_idx, g.n, s)[i, j]) < 1e-8


def _weights(seed, dims, l0):
    ws, lin = [], l0
    for k, lout in enumerate(dims, 1):
        ws.append(gcn.weight(seed, k, lin, lout))
        lin = lout
    return ws


def test_full_gradient_finite_differences(g):
    y = projection.project(g.row_ptr, g.col_idx, g.n, projection.MOD_FULL, 16, 2, 3)
    ws = _weights(3, [12, 8, 6], 16)
    loss, grads, g_y, _ = modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, y, ws)
    h = 1e-6
    rng = np.random.default_rng(2)
    for k in range(3):
        for _ in range(6):
            a, b = rng.integers(0, ws[k].shape[0]), rng.integers(0, ws[k].shape[1])
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[k][a, b] += h
            wm[k][a, b] -= h
            lp = modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, y, wp)[0]
            lm = modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, y, wm)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][a, b]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, a, b)
    for _ in range(6):
        i, j = rng.integers(0, g.n), rng.integers(0, 16)
        yp, ym = y.copy(), y.copy()
        yp[i, j] += h
        ym[i, j] -= h
        fd = (modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, yp, ws)[0]
              - modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, ym, ws)[0]) / (2 * h)
        assert abs(fd - g_y[i, j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_training_improves_modularity(g):
    """A few Adam steps lower the loss (sanity of sign and scale)."""
    y = projection.project(g.row_ptr, g.col_idx, g.n, projection.MOD_FULL, 16, 2, 3)
    ws = _weights(3, [16, 8], 16)
    ms = [np.zeros_like(w) for w in ws]
    vs = [np.zeros_like(w) for w in ws]
    l0 = None
    for t in range(1, 31):
        loss, grads, _, _ = modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, y, ws)
        l0 = loss if l0 is None else l0
        for k in range(len(ws)):
            ws[k], ms[k], vs[k] = modloss.adam_step(ws[k], ms[k], vs[k], grads[k], t)
    assert loss < l0


def test_adam_closed_form_first_step():
    w = np.array([1.0, -2.0]); g = np.array([0.5, -0.25])
    w1, m, v = modloss.adam_step(w, np.zeros(2), np.zeros(2), g, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> w - lr * sign(g) (up to eps)
    np.testing.assert_allclose(w1, w - 0.1 * np.sign(g), rtol=1e-6)


@pytest.fixture(scope="module")
def ball():
    """The N = 1,000 breadth-first ball of the training workload's graph
    (N = 200,000 DC-SBM), degrees recomputed inside the ball."""
    from synth import bfs_ball, make_workload
    g200k, _ = make_workload("n200k")
    return bfs_ball(g200k, 1000, root=0)


def test_gradient_fd_on_training_subgraph(ball):
    """Central finite differences (FP64, h = 1e-6) of the loss against the
    hand-written adjoint on the training workload's model (three layers of
    width 64, 64 softmax memberships), sampled entries of every W and of Y:
    relative error <= 1e-6."""
    g = ball
    y = projection.project(g.row_ptr, g.col_idx, g.n, projection.MOD_FULL, 64, 3, 0)
    ws = _weights(0, [64, 64, 64], 64)
    loss, grads, g_y, _ = modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, y, ws)
    h = 1e-6
    rng = np.random.default_rng(12)

    def lossw(w_list, yy):
        return modloss.loss_and_grads(g.row_ptr, g.col_idx, g.n, yy, w_list)[0]

    for k in range(3):
        for _ in range(5):
            a, b = rng.integers(0, 64), rng.integers(0, 64)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[k][a, b] += h
            wm[k][a, b] -= h
            fd = (lossw(wp, y) - lossw(wm, y)) / (2 * h)
            assert abs(fd - grads[k][a, b]) <= 1e-6 * max(abs(fd), 1e-3), (k, a, b, fd)
    for _ in range(5):
        i, j = rng.integers(0, g.n), rng.integers(0, 64)
        yp, ym = y.copy(), y.copy()
        yp[i, j] += h
        ym[i, j] -= h
        fd = (lossw(ws, yp) - lossw(ws, ym)) / (2 * h)
        assert abs(fd - g_y[i, j]) <= 1e-6 * max(abs(fd), 1e-3), (i, j, fd)
