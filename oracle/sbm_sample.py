"""Fast sampling of graphs from the degree-corrected SBM (Sec. IV, Alg. 2),
oracle side.

The model (Sec. II, SBM definition): node i in block c_i with degree
parameter theta_i; the count of edges between i and j is Poisson with mean
lambda_ij = theta_i theta_j Omega_{c_i c_j}, independently over pairs.  The
graph is undirected and unweighted: i and j are joined when their count is
positive, which happens with probability 1 - exp(-lambda_ij).

Alg. 2 visits the possible edges between blocks C_r and C_s (r <= s) as a
virtual |C_r| x |C_s| table and jumps from one positive entry to the next:
with the current position m and p ~ U(0, 1), the next positive entry is the
smallest t >= m with p > exp(-RangeSum(m, t)), RangeSum being the sum of the
lambdas from m to t (a prefix sum of theta gives it in O(1)), found by
binary search; no such t ends the table.

Readings (the paper leaves these open):
* the jump is run over each ROW of a block pair's table on its own -- row x
  of the (r, s) table holds the pairs (C_r[x], C_s[y]) -- which keeps the
  entries independent and the distribution exact while making every row an
  independent sequence (the rows are what the GPU runs in parallel);
* blocks list their nodes in increasing id; pairs r <= s; for r = s only
  the entries above the diagonal (y > x) are visited, so there are no self
  pairs and each unordered pair is visited once;
* p > exp(-S) is evaluated as E < S with E = -ln p (own FP64 ln), p the
  first word of Philox4x64-10 with key (seed, 0x30) and counter (pair id
  r K + s, x, jump, 0) as a uniform in (0, 1);
* RangeSum(m, t) over row x = (Omega_rs theta_{C_r[x]}) (P_s[t + 1] - P_s[m])
  with P_s the prefix sums of theta over C_s (FP64, accumulated left to
  right from 0); the binary search takes the smallest t in [m, |C_s|) with
  RangeSum(m, t) > E;
* a positive count's value (the zero-truncated Poisson of Alg. 2) is not
  drawn: only the support of A is used.

Pinned in ``tests/test_oracle_sampler.py``: edge frequencies over many seeds
against 1 - exp(-lambda_ij) pair by pair, expected edge counts against the
closed form, degenerate intensities, a direct per-pair Bernoulli sampler in
distribution, and CSR validity.
"""
import numpy as np

from . import fmath, philox

STREAM_SAMPLE = 0x30


def block_members(blocks, k):
    """Node ids of each block in increasing order."""
    blocks = np.asarray(blocks, dtype=np.int64)
    return [np.flatnonzero(blocks == r) for r in range(k)]


def prefix(theta, members):
    """P[0] = 0, P[y + 1] = P[y] + theta[members[y]] (left to right)."""
    out = np.zeros(members.size + 1, dtype=np.float64)
    acc = 0.0
    for y, i in enumerate(members):
        acc = acc + float(theta[i])
        out[y + 1] = acc
    return out


def sample_edges(theta, blocks, omega, seed):
    """Edges (i, j), one per sampled pair, in (r, s, x, jump) order."""
    theta = np.asarray(theta, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    k = omega.shape[0]
    members = block_members(blocks, k)
    pref = [prefix(theta, m) for m in members]
    key = np.array([seed, STREAM_SAMPLE], dtype=np.uint64)
    src, dst = [], []
    for r in range(k):
        for s in range(r, k):
            cr, cs, ps = members[r], members[s], pref[s]
            ns = cs.size
            if cr.size == 0 or ns == 0:
                continue
            pid = r * k + s
            # every row x of the table, all rows advanced together
            x = np.arange(cr.size, dtype=np.int64)
            lam = omega[r, s] * theta[cr]
            m = x + 1 if r == s else np.zeros(cr.size, dtype=np.int64)
            jump = np.zeros(cr.size, dtype=np.int64)
            live = m < ns
            while np.any(live):
                rows = np.flatnonzero(live)
                ctr = np.zeros((rows.size, 4), dtype=np.uint64)
                ctr[:, 0] = np.uint64(pid)
                ctr[:, 1] = x[rows].astype(np.uint64)
                ctr[:, 2] = jump[rows].astype(np.uint64)
                e = -fmath.ln(fmath.uniform52(philox.philox4x64(ctr, key)[:, 0]))
                jump[rows] += 1
                mm = m[rows]
                total = lam[rows] * (ps[ns] - ps[mm])
                hit = e < total
                live[rows[~hit]] = False
                rows, mm, e = rows[hit], mm[hit], e[hit]
                # smallest t in [m, ns) with lam (P[t + 1] - P[m]) > E
                lo, hi = mm.copy(), np.full(rows.size, ns - 1, dtype=np.int64)
                while np.any(lo < hi):
                    mid = (lo + hi) // 2
                    big = lam[rows] * (ps[mid + 1] - ps[mm]) > e
                    act = lo < hi
                    hi = np.where(act & big, mid, hi)
                    lo = np.where(act & ~big, mid + 1, lo)
                src.append(cr[x[rows]])
                dst.append(cs[lo])
                m[rows] = lo + 1
                live[rows] = lo + 1 < ns
    if not src:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    return np.concatenate(src), np.concatenate(dst)


def row_edges(theta, members, pref, omega, r, s, x, seed):
    """Columns (node ids) that row x of the (r, s) table joins to
    C_r[x], one jump at a time (the scalar form of ``sample_edges`` for
    single rows of large models)."""
    k = omega.shape[0]
    cs, ps = members[s], pref[s]
    ns = cs.size
    i = int(members[r][x])
    lam = float(omega[r, s]) * float(theta[i])
    key = np.array([seed, STREAM_SAMPLE], dtype=np.uint64)
    m = x + 1 if r == s else 0
    out, jump = [], 0
    while m < ns:
        ctr = np.array([[r * k + s, x, jump, 0]], dtype=np.uint64)
        e = float(-fmath.ln(fmath.uniform52(philox.philox4x64(ctr, key)[:, 0]))[0])
        jump += 1
        if not e < lam * (ps[ns] - ps[m]):
            break
        lo, hi = m, ns - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if lam * (ps[mid + 1] - ps[m]) > e:
                hi = mid
            else:
                lo = mid + 1
        out.append(int(cs[lo]))
        m = lo + 1
    return out


def sample_csr(theta, blocks, omega, seed):
    """The sampled graph as a symmetric CSR (int64 row_ptr, int64 col_idx,
    rows sorted)."""
    n = np.asarray(theta).size
    a, b = sample_edges(theta, blocks, omega, seed)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols
