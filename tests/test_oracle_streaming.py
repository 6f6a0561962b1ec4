"""Pins of the streaming update (Sec. III-D): the incremental levels equal a
full recomputation on the new graph (projection levels bit for bit, GCN
layers to rounding), levels outside their hop balls do not change under the
NCut operator and do change under the modularity operators, hop distances
equal scipy's shortest paths, and the merged CSR is valid and rejects
malformed edge sets."""
import numpy as np
import pytest

from oracle import graph as ograph
from oracle import streaming
from synth.dcsbm import dcsbm


@pytest.fixture(scope="module")
def base():
    g = dcsbm(1500, 6, seed=4, d_min=3.0, d_max=30.0)
    return g


def new_edges(g, m, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    have = set((rows * g.n + g.col_idx).tolist())
    out = set()
    while len(out) < m:
        a, b = (int(v) for v in rng.integers(0, g.n, 2))
        if a == b:
            continue
        a, b = min(a, b), max(a, b)
        if a * g.n + b in have or (a, b) in out:
            continue
        out.add((a, b))
    e = np.array(sorted(out))
    return e[:, 0], e[:, 1]


def test_add_edges_valid_and_rejects(base):
    g = base
    s, d = new_edges(g, 40, 1)
    rp, ci = streaming.add_edges(g.row_ptr, g.col_idx, g.n, s, d)
    ograph.validate_csr(rp.astype(np.int32), ci.astype(np.int32), g.n)
    assert rp[-1] == g.nnz + 80
    for a, b in zip(s, d):
        assert b in ci[rp[a]:rp[a + 1]] and a in ci[rp[b]:rp[b + 1]]
    with pytest.raises(ValueError):
        streaming.add_edges(g.row_ptr, g.col_idx, g.n, [3], [3])
    with pytest.raises(ValueError):
        streaming.add_edges(g.row_ptr, g.col_idx, g.n, [0], [g.n])
    j = int(g.col_idx[g.row_ptr[5]])
    with pytest.raises(ValueError):
        streaming.add_edges(g.row_ptr, g.col_idx, g.n, [j], [5])
    with pytest.raises(ValueError):
        streaming.add_edges(g.row_ptr, g.col_idx, g.n, [s[0], d[0]], [d[0], s[0]])


def test_hop_distance_matches_library(base):
    g = base
    rng = np.random.default_rng(3)
    src = rng.choice(g.n, 5, replace=False)
    for radius in (0, 1, 3, 6):
        a = streaming.hop_distance(g.row_ptr, g.col_idx, g.n, src, radius)
        b = streaming.hop_distance_library(g.row_ptr, g.col_idx, g.n, src, radius)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("normalize_input", [False, True])
def test_ncut_update_equals_full_and_is_local(base, normalize_input):
    g = base
    q, dims, L, seed = 2, [16, 8], 16, 7
    prev = streaming.levels(g.row_ptr, g.col_idx, g.n, 0, L, q, dims, seed, normalize_input)
    s, d = new_edges(g, 3, 2)
    rp, ci = streaming.add_edges(g.row_ptr, g.col_idx, g.n, s, d)
    vprime = np.unique(np.concatenate([s, d]))
    inc, sizes = streaming.update(prev, rp, ci, g.n, 0, q, dims, seed, vprime, normalize_input)
    full = streaming.levels(rp, ci, g.n, 0, L, q, dims, seed, normalize_input)
    for t in range(q + 1):
        assert np.array_equal(inc["y"][t], full["y"][t])      # sparse rows: same sums
    assert np.allclose(inc["h0"], full["h0"], rtol=0, atol=1e-15)
    for a, b in zip(inc["h"], full["h"]):
        assert np.allclose(a, b, rtol=0, atol=1e-14)
    # locality: outside its ball a level is the old graph's, inside it moves
    dist = streaming.hop_distance(rp, ci, g.n, vprime, q + len(dims))
    assert sizes == [int(np.sum(dist <= t)) for t in range(1, q + len(dims) + 1)]
    assert sizes[-1] < g.n
    for t in range(1, q + 1):
        out = dist > t
        assert np.array_equal(full["y"][t][out], prev["y"][t][out])
        assert not np.allclose(full["y"][t][dist == t], prev["y"][t][dist == t], rtol=0, atol=0)
    for k in range(1, len(dims) + 1):
        out = dist > q + k
        assert np.allclose(full["h"][k - 1][out], prev["h"][k - 1][out], rtol=0, atol=1e-15)


@pytest.mark.parametrize("op", [1, 2])
def test_modularity_levels_change_everywhere(base, op):
    """Under Eq. 4 and Q~ one new edge changes 2e and with it rows far
    outside the hop balls, so the update recomputes every row."""
    g = base
    q, dims, L, seed = 2, [8], 8, 3
    prev = streaming.levels(g.row_ptr, g.col_idx, g.n, op, L, q, dims, seed)
    s, d = new_edges(g, 1, 5)
    rp, ci = streaming.add_edges(g.row_ptr, g.col_idx, g.n, s, d)
    vprime = np.concatenate([s, d])
    full = streaming.levels(rp, ci, g.n, op, L, q, dims, seed)
    dist = streaming.hop_distance(rp, ci, g.n, vprime, q + len(dims))
    far = dist > q
    changed = np.any(full["y"][q][far] != prev["y"][q][far], axis=1)
    assert changed.mean() > 0.5
    inc, sizes = streaming.update(prev, rp, ci, g.n, op, q, dims, seed, vprime)
    assert sizes == [g.n] * (q + len(dims))
    for t in range(q + 1):
        assert np.array_equal(inc["y"][t], full["y"][t])
    for a, b in zip(inc["h"], full["h"]):
        assert np.allclose(a, b, rtol=0, atol=1e-14)
