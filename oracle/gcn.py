"""Random, untrained GCN embedding (oracle side).

Sec. III-B, Eq. 6: Z^(k) = tanh( D_hat^-1/2 A_hat D_hat^-1/2 Z^(k-1) W^(k) ),
A_hat = A + I, D_hat its degree matrix, Z^(0) = Y, no bias term.  Each layer's
output is L2-normalised row by row before the next layer, and the normalised
output of the last layer is the embedding Z.  The weights are random and never
trained (Sec. III-B: one feed-forward pass of a randomly initialised GNN).

Readings:
* W^(k)_ab ~ N(0, 1/L_{k-1}) (std L_{k-1}^-1/2), drawn from Philox with key
  (seed, 0x10 + k), counter (a, col_block), FP32-rounded like Theta;
* Y is not normalised before layer 1 unless ``normalize_input`` is set;
* a zero row is divided by max(||z||, 1e-12) and stays zero;
* (A_hat Z) W is evaluated in that order.
"""
import numpy as np
import scipy.sparse as sp

from . import philox
from .graph import adjacency, degrees
from .projection import gaussian_matrix


def gcn_operator(row_ptr, col_idx, n):
    """A_hat_n = D_hat^-1/2 (A + I) D_hat^-1/2 (Eq. 6)."""
    a = adjacency(row_ptr, col_idx, n) + sp.identity(n, format="csr")
    s = 1.0 / np.sqrt(degrees(row_ptr).astype(np.float64) + 1.0)
    return (sp.diags(s) @ a @ sp.diags(s)).tocsr()


def weight(seed, k, l_in, l_out):
    """W^(k) in R^{L_{k-1} x L_k}, std L_{k-1}^-1/2."""
    return gaussian_matrix(seed, philox.STREAM_W_BASE + k, l_in, l_out,
                           1.0 / np.sqrt(float(l_in)))


def row_normalize(z):
    nrm = np.sqrt(np.sum(z * z, axis=1))
    return z / np.maximum(nrm, 1e-12)[:, None]


def embed(row_ptr, col_idx, n, y, dims, seed, normalize_input=False, weights=None):
    """Forward pass of the random GCN.  dims = [L_1, ..., L_n] (d = L_n)."""
    ahat = gcn_operator(row_ptr, col_idx, n)
    h = np.asarray(y, dtype=np.float64)
    if normalize_input:
        h = row_normalize(h)
    l_in = h.shape[1]
    for k, l_out in enumerate(dims, start=1):
        w = weight(seed, k, l_in, l_out) if weights is None else weights[k - 1]
        p = ahat @ h
        z = np.tanh(p @ w)
        h = row_normalize(z)
        l_in = l_out
    return h
