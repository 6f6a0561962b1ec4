"""Gaussian random projection of the GP objectives (oracle side).

Sec. III-A: X is the structural component of NCut (M = D^-1/2 A D^-1/2,
from the normalised Laplacian of Eq. 2) or of modularity (Eq. 4); features are
Y = X Theta with Theta_ir Gaussian, zero mean, spread L^-0.5 (Eq. 5).

Readings (documented in the design notes):
* the spread L^-0.5 is the standard deviation (variance 1/L), the
  Johnson-Lindenstrauss normalisation;
* Y = X^q Theta, i.e. q successive products; q = 1 is Eq. 5 exactly;
* X is one of
    NCUT         M, with D^-1/2 = 0 for an isolated node;
    MOD_FULL     the full modularity matrix B = A - d d^T / 2e (Eq. 4),
                 applied as A Y - d (d^T Y) / 2e so B is never formed;
    MOD_REDUCED  the paper's reduced matrix Q~ (Q masked to the edge set,
                 Sec. III-A), entries 1 - d_i d_j / 2e on edges.
* Theta is drawn from Philox4x64-10 with key (seed, 0x10), counter
  (row, col_block, 0, 0); each block gives four Box-Muller normals for
  columns 4*col_block .. 4*col_block+3; the value is sigma * z rounded to FP32
  (round to nearest even) and then used in FP64, so both sides of the parity
  check hold the identical matrix.
"""
import numpy as np
import scipy.sparse as sp

from . import fmath, philox
from .graph import adjacency, degrees, two_e

NCUT, MOD_FULL, MOD_REDUCED = 0, 1, 2


def gaussian_matrix(seed, stream, rows, cols, sigma):
    """FP32-rounded sigma * N(0,1) matrix [rows, cols], returned as float64."""
    cb = (cols + 3) // 4
    blk = philox.block_grid(seed, stream, rows, cb)
    z = fmath.normals_from_block(blk).reshape(rows, cb * 4)[:, :cols]
    return (sigma * z).astype(np.float32).astype(np.float64)


def theta(seed, n, L):
    """Theta in R^{N x L}, std L^-1/2 (Eq. 5)."""
    sigma = 1.0 / np.sqrt(float(L))
    return gaussian_matrix(seed, philox.STREAM_THETA, n, L, sigma)


def ncut_operator(row_ptr, col_idx, n):
    """M = D^-1/2 A D^-1/2 (Sec. III-A), D^-1/2 = 0 for isolated nodes."""
    a = adjacency(row_ptr, col_idx, n)
    d = degrees(row_ptr).astype(np.float64)
    s = np.where(d > 0, 1.0 / np.sqrt(np.maximum(d, 1.0)), 0.0)
    return sp.diags(s) @ a @ sp.diags(s)


def reduced_modularity_operator(row_ptr, col_idx, n):
    """Q~: Q_ij = A_ij - d_i d_j / 2e kept on the edge set only (Sec. III-A)."""
    a = adjacency(row_ptr, col_idx, n).tocoo()
    d = degrees(row_ptr).astype(np.float64)
    m2 = float(two_e(row_ptr))
    vals = 1.0 - d[a.row] * d[a.col] / m2
    return sp.csr_matrix((vals, (a.row, a.col)), shape=(n, n))


def apply_modularity(a, d, m2, y):
    """B y = A y - d (d^T y) / 2e (Eq. 4), B never formed."""
    return a @ y - np.outer(d, d @ y) / m2


def project(row_ptr, col_idx, n, op, L, q, seed, theta_in=None):
    """Y = X^q Theta in FP64.  Returns Y [n, L]."""
    y = theta(seed, n, L) if theta_in is None else np.asarray(theta_in, np.float64)
    if op == NCUT:
        m = ncut_operator(row_ptr, col_idx, n)
        for _ in range(q):
            y = m @ y
    elif op == MOD_FULL:
        a = adjacency(row_ptr, col_idx, n)
        d = degrees(row_ptr).astype(np.float64)
        m2 = float(two_e(row_ptr))
        for _ in range(q):
            y = apply_modularity(a, d, m2, y)
    elif op == MOD_REDUCED:
        qr = reduced_modularity_operator(row_ptr, col_idx, n)
        for _ in range(q):
            y = qr @ y
    else:
        raise ValueError("unknown operator")
    return np.asarray(y)
