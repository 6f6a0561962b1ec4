"""CSR input checks and degree statistics (oracle side).

The paper studies undirected, unweighted graphs whose adjacency matrix A is
symmetric with entries in {0, 1} (Sec. II, problem statement).  Degrees and the
edge count e enter NCut (Eq. 1-2: D = diag(deg)), modularity (Eq. 3-4: 2e) and
the GCN operator (Eq. 6: A_hat = A + I, D_hat its degree matrix).

Self-pairs are not edges here: A_hat adds the identity explicitly (Eq. 6), so
a stored diagonal entry is rejected.  Pinned against scipy.sparse / networkx
degrees in ``tests/test_oracle_graph.py``.
"""
import numpy as np
import scipy.sparse as sp


class CSRError(ValueError):
    pass


def validate_csr(row_ptr, col_idx, n):
    """Raise CSRError unless (row_ptr, col_idx) is a valid symmetric,
    sorted, duplicate-free, loop-free CSR adjacency of an n-node graph."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    if row_ptr.shape != (n + 1,):
        raise CSRError("row_ptr must have n+1 entries")
    if row_ptr[0] != 0 or row_ptr[-1] != col_idx.size:
        raise CSRError("row_ptr must start at 0 and end at nnz")
    if np.any(np.diff(row_ptr) < 0):
        raise CSRError("row_ptr must be non-decreasing")
    if col_idx.size and (col_idx.min() < 0 or col_idx.max() >= n):
        raise CSRError("column index out of range")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    if np.any(rows == col_idx):
        raise CSRError("self-loop")
    # strictly increasing columns inside every row
    same_row = rows[1:] == rows[:-1]
    if np.any(same_row & (col_idx[1:] <= col_idx[:-1])):
        raise CSRError("columns must be sorted and unique within a row")
    a = sp.csr_matrix((np.ones(col_idx.size), col_idx, row_ptr), shape=(n, n))
    if (a != a.T).nnz != 0:
        raise CSRError("adjacency must be symmetric")


def degrees(row_ptr):
    """deg(v_i) = number of stored neighbours (int64)."""
    return np.diff(np.asarray(row_ptr, dtype=np.int64))


def two_e(row_ptr):
    """2e = sum of degrees = number of stored CSR entries (int64)."""
    return int(np.asarray(row_ptr, dtype=np.int64)[-1])


def adjacency(row_ptr, col_idx, n):
    """A as a float64 scipy CSR matrix with unit values."""
    return sp.csr_matrix(
        (np.ones(len(col_idx), dtype=np.float64),
         np.asarray(col_idx, dtype=np.int64),
         np.asarray(row_ptr, dtype=np.int64)),
        shape=(n, n))
