"""Merge-path SpMM (raft_spmm_merge): every operator and width against the
FP64 oracle per column, on a heavy-tailed graph with ragged tiles, on a graph
whose hub row spans many path ranges next to empty rows, and against the
row-split kernel."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import graph as ograph
from oracle import projection
from synth import dcsbm
from synth.dcsbm import edges_to_csr

pytestmark = pytest.mark.gpu

COL_TOL = 1e-5


@pytest.fixture(scope="module")
def api_mod():
    from paper_2312_01560_amd import api
    return api


@pytest.fixture(scope="module")
def ctx(api_mod):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = api_mod.Context(0)
    yield c
    c.close()


def col_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def oracle_step(rp, ci, n, op, x):
    if op == 0:
        return projection.ncut_operator(rp, ci, n) @ x
    if op == 1:
        a = ograph.adjacency(rp, ci, n)
        d = ograph.degrees(rp).astype(float)
        return projection.apply_modularity(a, d, float(ograph.two_e(rp)), x)
    if op == 2:
        return projection.reduced_modularity_operator(rp, ci, n) @ x
    return ogcn.gcn_operator(rp, ci, n) @ x


def hub_graph():
    """A hub joined to 3,000 of 5,000 nodes (its row spans many 256-item
    ranges), a sparse random part, and every 7th node isolated."""
    n = 5000
    rng = np.random.default_rng(9)
    src = list(np.zeros(3000, dtype=np.int64))
    dst = list(rng.choice(np.arange(1, n), 3000, replace=False))
    a = rng.integers(1, n, 8000)
    b = rng.integers(1, n, 8000)
    keep = (a != b) & (a % 7 != 0) & (b % 7 != 0)
    src += list(a[keep])
    dst += list(b[keep])
    src, dst = np.asarray(src), np.asarray(dst)
    keep = (src % 7 != 0) | (src == 0)
    keep &= (dst % 7 != 0) | (dst == 0)
    rp, ci = edges_to_csr(n, src[keep], dst[keep])
    return n, rp, ci


@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [16, 64, 128, 256])
def test_merge_against_oracle(ctx, api_mod, op, L):
    g0 = dcsbm(3001, 9, gamma=2.2, d_min=5, d_max=400, rho=2.0, seed=11)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    x = np.random.default_rng(L + op).standard_normal((g0.n, L)).astype(np.float32)
    got = api_mod.spmm_merge(ctx, g, op, torch.from_numpy(x).cuda())
    row = api_mod.spmm(ctx, g, op, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    ref = oracle_step(g0.row_ptr, g0.col_idx, g0.n, op, x.astype(np.float64))
    assert col_err(got.cpu().numpy(), ref).max() < COL_TOL
    assert col_err(got.cpu().numpy(), row.cpu().numpy().astype(np.float64)).max() < COL_TOL
    g.close()


@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_merge_hub_and_empty_rows(ctx, api_mod, op):
    n, rp, ci = hub_graph()
    assert np.diff(rp)[0] >= 2500 and np.sum(np.diff(rp) == 0) > 500
    g = api_mod.Graph(ctx, rp, ci)
    x = np.random.default_rng(3).standard_normal((n, 64)).astype(np.float32)
    got = api_mod.spmm_merge(ctx, g, op, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    ref = oracle_step(rp, ci, n, op, x.astype(np.float64))
    assert col_err(got.cpu().numpy(), ref).max() < COL_TOL
    # empty rows: zero under NCut and modularity, the self term under the GCN
    empty = np.flatnonzero(np.diff(rp) == 0)
    y = got.cpu().numpy()
    if op in (0, 2):
        assert np.all(y[empty] == 0)
    elif op == 3:
        assert np.array_equal(y[empty], x[empty])     # (0 + 1 * x) * 1
    g.close()


def test_merge_deterministic(ctx, api_mod):
    g0 = dcsbm(20011, 17, gamma=2.1, d_min=3, d_max=2000, rho=2.0, seed=5)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    x = torch.randn(g0.n, 128, device="cuda")
    a = api_mod.spmm_merge(ctx, g, 0, x)
    b = api_mod.spmm_merge(ctx, g, 0, x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    g.close()
