"""Parity of the training path (relaxed modularity loss, hand-written GCN
adjoint, Adam) with the FP64 oracle, whose gradients are pinned by central
finite differences in tests/test_oracle_modloss.py (also on the N = 1,000
ball of the training workload's graph).

Bars: forward values (logits U, saved layer outputs, memberships S) within
1e-5 relative Frobenius error per column; gradients element by element:
|g - g_ref| <= 1e-4 * mag, where mag is the same adjoint evaluated over the
absolute values of every term (each gradient entry is a sum of products;
mag is the sum of their absolute values, the quantity an FP32 evaluation's
rounding error is proportional to).  A wrong term, row, column or sign
gives an error of the order of mag itself."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import graph as ograph
from oracle import modloss, projection, scores
from synth import dcsbm

pytestmark = pytest.mark.gpu

COL_TOL = 1e-5
GRAD_C = 1e-4


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2312_01560_amd import api
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def graph():
    return dcsbm(1500, 8, gamma=2.4, d_min=6, d_max=120, rho=2.5, seed=21)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def col_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    nrm = np.linalg.norm(ref, axis=0)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(nrm, 1e-300)


def assert_within_mag(got, ref, mag, what):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bound = GRAD_C * mag + 1e-30
    worst = np.unravel_index(np.argmax(err / bound), err.shape)
    assert np.all(err <= bound), (what, worst, err[worst], mag[worst], ref[worst])


def grad_s_mag(rp, ci, n, s):
    """|terms| of dloss/dS = -(A S - d (d^T S)/2e)/e."""
    a = ograph.adjacency(rp, ci, n)
    d = ograph.degrees(rp).astype(np.float64)
    m2 = float(ograph.two_e(rp))
    sa = np.abs(s)
    return (a @ sa + np.outer(d, d @ sa) / m2) / (m2 / 2.0)


def softmax_backward_mag(s, g_s, g_s_mag):
    """|terms| of S o (G_S - rowsum(G_S o S)), given |terms| of G_S."""
    return s * (g_s_mag + np.sum(g_s_mag * s, axis=1, keepdims=True))


def adjoint_mags(rp, ci, n, weights, inputs, g_u_mag):
    """The adjoint of the training forward (the oracle's backward) evaluated
    over absolute values: magnitudes of dL/dW^(k) and dL/dY."""
    ahat = ogcn.gcn_operator(rp, ci, n)             # non-negative
    last = len(weights) - 1
    mags = [None] * len(weights)
    mg = g_u_mag
    for k in range(last, -1, -1):
        h = inputs[k]
        p = ahat @ h
        w = weights[k]
        if k == last:
            mgu = mg
        else:
            z = np.tanh(p @ w)
            nrm = np.maximum(np.sqrt(np.sum(z * z, axis=1)), 1e-12)[:, None]
            zh = np.abs(z / nrm)
            mgz = (mg + zh * np.sum(zh * mg, axis=1, keepdims=True)) / nrm
            mgu = mgz * np.abs(1.0 - z * z)
        mags[k] = (ahat @ np.abs(h)).T @ mgu
        mg = ahat @ (mgu @ np.abs(w).T)
    return mags, mg


def to_np(t):
    return t.detach().cpu().double().numpy()


def _setup(ctx, g0, dims, seed=4):
    from paper_2312_01560_amd import api
    from paper_2312_01560_amd.train import Trainer
    g = api.Graph(ctx, g0.row_ptr, g0.col_idx)
    y = api.project(ctx, g, api.Config(op=0, proj_dim=dims[0], q=2, layer_dims=[dims[0]]))
    ws = [api.gaussian(ctx, seed, 0x10 + k + 1, dims[k], dims[k + 1], dims[k] ** -0.5)
          for k in range(len(dims) - 1)]
    return g, y, ws, Trainer(ctx, g, dims)


def check_forward_backward(ctx, g0, dims, seed):
    """Forward (per column at 1e-5), loss, and every gradient element by
    element, each GPU stage against the oracle applied to the GPU's own
    inputs of that stage."""
    g, y, ws, tr = _setup(ctx, g0, dims, seed)
    rp, ci, n = g0.row_ptr, g0.col_idx, g0.n
    U, saved = tr.forward(y, ws)
    S, loss = tr.modloss_forward(U)
    GU = tr.modloss_backward(S)
    GW, GH0 = tr.backward(y, ws, saved, GU, want_h0=True)
    torch.cuda.synchronize()
    y64 = to_np(y)
    w64 = [to_np(w) for w in ws]
    u_ref, inputs = modloss.forward(rp, ci, n, y64, w64)
    assert col_err(to_np(U), u_ref).max() < COL_TOL
    for k, h in enumerate(saved):
        assert col_err(to_np(h), inputs[k + 1]).max() < COL_TOL, k
    s64 = to_np(S)
    assert col_err(s64, modloss.softmax_rows(to_np(U))).max() < COL_TOL
    l_ref = modloss.loss_of_s(rp, ci, n, s64)
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * abs(l_ref) + 1e-9
    g_s = modloss.grad_s(rp, ci, n, s64)
    gu_ref = modloss.softmax_backward(s64, g_s)
    assert_within_mag(to_np(GU), gu_ref, softmax_backward_mag(s64, g_s, grad_s_mag(rp, ci, n, s64)),
                      "dL/dU")
    gu64 = to_np(GU)
    layer_in = [y64] + [to_np(h) for h in saved]
    gw_ref, gy_ref = modloss.backward(rp, ci, n, w64, layer_in, gu64)
    mags, gy_mag = adjoint_mags(rp, ci, n, w64, layer_in, np.abs(gu64))
    for k in range(len(ws)):
        assert_within_mag(to_np(GW[k]), gw_ref[k], mags[k], f"dL/dW{k + 1}")
    assert_within_mag(to_np(GH0), gy_ref, gy_mag, "dL/dY")
    return g, y, ws


@pytest.mark.parametrize("dims", [[64, 64, 64, 64], [32, 64, 16], [128, 64]])
def test_forward_backward_vs_oracle(ctx, graph, dims):
    check_forward_backward(ctx, graph, dims, 4)


def test_gradients_on_training_subgraph_vs_fd(ctx):
    """The training workload's model (3 x 64, 64 memberships) on the
    N = 1,000 breadth-first ball of its graph: every gradient element against
    the oracle's adjoint, and sampled entries of dL/dW against FP64 central
    finite differences of the oracle's loss at the GPU's weights."""
    from synth import bfs_ball, make_workload
    g200k, _ = make_workload("n200k")
    g0 = bfs_ball(g200k, 1000, root=0)
    dims = [64, 64, 64, 64]
    g, y, ws = check_forward_backward(ctx, g0, dims, 0)
    from paper_2312_01560_amd.train import Trainer
    tr = Trainer(ctx, g, dims)
    U, saved = tr.forward(y, ws)
    S, _ = tr.modloss_forward(U)
    GW, _ = tr.backward(y, ws, saved, tr.modloss_backward(S))
    torch.cuda.synchronize()
    y64 = to_np(y)
    w64 = [to_np(w) for w in ws]
    rp, ci, n = g0.row_ptr, g0.col_idx, g0.n
    _, g_ref, _, s_ref = modloss.loss_and_grads(rp, ci, n, y64, w64)
    _, inputs = modloss.forward(rp, ci, n, y64, w64)
    g_s = modloss.grad_s(rp, ci, n, s_ref)
    mags, _ = adjoint_mags(rp, ci, n, w64, inputs,
                           softmax_backward_mag(s_ref, g_s, grad_s_mag(rp, ci, n, s_ref)))
    h = 1e-6
    rng = np.random.default_rng(3)
    for k in range(3):
        for _ in range(4):
            a, b = rng.integers(0, 64), rng.integers(0, 64)
            wp = [w.copy() for w in w64]
            wm = [w.copy() for w in w64]
            wp[k][a, b] += h
            wm[k][a, b] -= h
            fd = (modloss.loss_and_grads(rp, ci, n, y64, wp)[0]
                  - modloss.loss_and_grads(rp, ci, n, y64, wm)[0]) / (2 * h)
            assert abs(fd - g_ref[k][a, b]) <= 1e-6 * max(abs(fd), 1e-3)
            assert abs(to_np(GW[k])[a, b] - fd) <= GRAD_C * mags[k][a, b] + 1e-6 * abs(fd), (k, a, b)


def test_autograd_end_to_end_matches_oracle(ctx, graph):
    from paper_2312_01560_amd.train import RaftGCN, RaftModLoss
    dims = [64, 64, 64, 64]
    g, y, ws, tr = _setup(ctx, graph, dims, seed=9)
    params = [w.clone().requires_grad_(True) for w in ws]
    U = RaftGCN.apply(tr, y, *params)
    loss = RaftModLoss.apply(tr, U)
    (2.0 * loss).backward()
    l_ref, g_ref, _, _ = modloss.loss_and_grads(graph.row_ptr, graph.col_idx, graph.n, to_np(y),
                                                [to_np(w) for w in ws])
    assert abs(loss.item() - l_ref) <= 1e-5 * abs(l_ref)
    rp, ci, n = graph.row_ptr, graph.col_idx, graph.n
    w64 = [to_np(w) for w in ws]
    _, inputs = modloss.forward(rp, ci, n, to_np(y), w64)
    _, _, _, s_ref = modloss.loss_and_grads(rp, ci, n, to_np(y), w64)
    g_s = modloss.grad_s(rp, ci, n, s_ref)
    mags, _ = adjoint_mags(rp, ci, n, w64, inputs,
                           softmax_backward_mag(s_ref, g_s, grad_s_mag(rp, ci, n, s_ref)))
    for k, p in enumerate(params):
        assert_within_mag(to_np(p.grad), 2.0 * g_ref[k], 2.0 * mags[k], f"autograd dW{k + 1}")


def test_adam_matches_oracle(ctx, graph):
    from paper_2312_01560_amd.train import Trainer
    from paper_2312_01560_amd import api
    g = api.Graph(ctx, graph.row_ptr, graph.col_idx)
    tr = Trainer(ctx, g, [16, 16])
    rng = np.random.default_rng(0)
    w = rng.standard_normal(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda")
    mt = torch.zeros_like(wt)
    vt = torch.zeros_like(wt)
    for step in range(1, 6):
        grad = rng.standard_normal(1000)
        tr.adam(wt, mt, vt, torch.tensor(grad, dtype=torch.float32, device="cuda"), step)
        w, m, v = modloss.adam_step(w, m, v, grad.astype(np.float32).astype(np.float64), step)
    np.testing.assert_allclose(to_np(wt), w, rtol=1e-6, atol=1e-7)


def test_training_lowers_loss_and_partitions(ctx, graph):
    """20 Adam steps lower the loss; the hard partition of the trained model
    scores its modularity exactly as the oracle does (Eq. 3)."""
    from paper_2312_01560_amd import api
    dims = [64, 64, 64]
    g, y, ws, tr = _setup(ctx, graph, dims, seed=5)
    params = [w.clone() for w in ws]
    ms = [torch.zeros_like(w) for w in ws]
    vs = [torch.zeros_like(w) for w in ws]
    losses = []
    for step in range(1, 21):
        U, saved = tr.forward(y, params)
        S, loss = tr.modloss_forward(U)
        losses.append(loss.item())
        GW, _ = tr.backward(y, params, saved, tr.modloss_backward(S))
        for k in range(len(params)):
            tr.adam(params[k], ms[k], vs[k], GW[k], step)
    assert losses[-1] < losses[0]
    lab = torch.argmax(S, dim=1).to(torch.uint8)[:, None].contiguous()
    k = int(lab.max().item()) + 1
    mod, _ = api.score(ctx, g, lab, [max(k, 1)])
    ref = scores.modularity(graph.row_ptr, graph.col_idx, lab[:, 0].cpu().numpy().astype(np.int64), max(k, 1))
    assert to_np(mod)[0] == ref


def test_forward_backward_full_size_n200k(ctx):
    """The training workload's size (N = 200,000, GCN 3 x 64): logits,
    saved layer outputs and memberships per column, the loss, and dL/dU,
    every weight gradient and dL/dY element by element against the FP64
    oracle."""
    from synth import make_workload
    g0, _ = make_workload("n200k")
    check_forward_backward(ctx, g0, [64, 64, 64, 64], 6)
