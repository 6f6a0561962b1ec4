"""Relaxed modularity loss and the adjoint of the GCN (oracle side).

Not in the paper, which never trains its GCN (Sec. III-B: one feed-forward
pass of a randomly initialised GNN); the weights W^(k) are nevertheless
trainable parameters of Eq. 6.  The loss relaxes the matrix form of
modularity (Eq. 4): with hard memberships H, tr(H^T B H)/2e is the modularity
of Eq. 3; replacing H by row-softmax assignments S gives

    loss = -tr(S^T B S) / 2e,   B = A - d d^T / 2e (never formed),
    tr(S^T B S) = sum_i S_i . (A S)_i - ||d^T S||^2 / 2e.

Model for training: hidden layers as Eq. 6 (tanh, row L2 normalisation);
the last layer is linear, U = (A_hat_n H) W, and S = softmax_rows(U).

Adjoint (hand-derived):
    dloss/dS = -(B S) / e
    softmax:      G_U = S o (G_S - rowsum(G_S o S))
    linear layer: G_W = P^T G_U,  G_P = G_U W^T,  G_H = A_hat_n G_P (A_hat_n symmetric)
    hidden layer: Zh = Z / ||Z||:  G_Z = (G_Zh - Zh (Zh . G_Zh)) / ||Z||,
                  G_U = G_Z o (1 - Z^2), then as the linear layer.

Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pinned in ``tests/test_oracle_modloss.py`` by central finite differences in
FP64 and by the closed form loss(one-hot S) = -Mod (Eq. 3).
"""
import numpy as np

from .gcn import gcn_operator, row_normalize
from .graph import adjacency, degrees, two_e


def softmax_rows(u):
    u = np.asarray(u, dtype=np.float64)
    e = np.exp(u - u.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def apply_b(row_ptr, col_idx, n, s):
    a = adjacency(row_ptr, col_idx, n)
    d = degrees(row_ptr).astype(np.float64)
    m2 = float(two_e(row_ptr))
    return a @ s - np.outer(d, d @ s) / m2


def loss_of_s(row_ptr, col_idx, n, s):
    """-tr(S^T B S) / 2e."""
    m2 = float(two_e(row_ptr))
    return -float(np.sum(s * apply_b(row_ptr, col_idx, n, s))) / m2


def grad_s(row_ptr, col_idx, n, s):
    """d loss / d S = -(B S) / e."""
    e = float(two_e(row_ptr)) / 2.0
    return -apply_b(row_ptr, col_idx, n, s) / e


def softmax_backward(s, g_s):
    return s * (g_s - np.sum(g_s * s, axis=1, keepdims=True))


def forward(row_ptr, col_idx, n, y, weights):
    """Training forward: returns (U, layer inputs H^(0..L-1))."""
    ahat = gcn_operator(row_ptr, col_idx, n)
    h = np.asarray(y, dtype=np.float64)
    inputs = []
    for k, w in enumerate(weights):
        inputs.append(h)
        p = ahat @ h
        u = p @ w
        if k == len(weights) - 1:
            return u, inputs
        h = row_normalize(np.tanh(u))
    raise ValueError("no layers")


def backward(row_ptr, col_idx, n, weights, inputs, g_u):
    """Adjoint of forward: returns (grads of W (list), grad of the input Y).
    Activations are recomputed from the stored layer inputs."""
    ahat = gcn_operator(row_ptr, col_idx, n)
    grads = [None] * len(weights)
    g = np.asarray(g_u, dtype=np.float64)
    last = len(weights) - 1
    for k in range(last, -1, -1):
        p = ahat @ inputs[k]
        w = weights[k]
        if k == last:
            gu = g
        else:
            z = np.tanh(p @ w)
            nrm = np.maximum(np.sqrt(np.sum(z * z, axis=1)), 1e-12)[:, None]
            zh = z / nrm
            gz = (g - zh * np.sum(zh * g, axis=1, keepdims=True)) / nrm
            gu = gz * (1.0 - z * z)
        grads[k] = p.T @ gu
        g = ahat @ (gu @ w.T)
    return grads, g


def loss_and_grads(row_ptr, col_idx, n, y, weights):
    u, inputs = forward(row_ptr, col_idx, n, y, weights)
    s = softmax_rows(u)
    loss = loss_of_s(row_ptr, col_idx, n, s)
    g_u = softmax_backward(s, grad_s(row_ptr, col_idx, n, s))
    grads, g_y = backward(row_ptr, col_idx, n, weights, inputs, g_u)
    return loss, grads, g_y, s


def adam_step(w, m, v, g, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
