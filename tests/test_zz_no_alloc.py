"""The allocation-free SpMM entry point (raft_spmm_noalloc) against raft_spmm
with a caller workspace: identical results, bit for bit, on two calls in a
row, the second on a smaller graph (the fixed scratch then holds the first
call's partials beyond what the second writes)."""
import numpy as np
import pytest
import torch

from synth import dcsbm

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("op", [1, 0, 2, 3])
@pytest.mark.parametrize("L", [64, 128])
def test_noalloc_matches_workspace_entry(ctx, api_mod, op, L):
    graphs = [dcsbm(20011, 17, gamma=2.3, d_min=5, d_max=400, rho=2.0, seed=21),
              dcsbm(3001, 9, gamma=2.2, d_min=5, d_max=300, rho=2.0, seed=22)]
    for step, g0 in enumerate(graphs):
        print(f"noalloc op={op} L={L} call={step} n={g0.n}", flush=True)
        g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
        x = torch.from_numpy(np.random.default_rng(5 + step).standard_normal(
            (g0.n, L)).astype(np.float32)).cuda()
        ref = api_mod.spmm(ctx, g, op, x)
        got = torch.full((g0.n, L), float("nan"), dtype=torch.float32, device="cuda")
        api_mod.spmm_noalloc(ctx, g, op, x, got)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert torch.equal(got, ref), (op, L, step)
        g.close()


def test_noalloc_rejects_oversized(ctx, api_mod):
    """MOD_FULL partials beyond the fixed scratch: a clear error, no launch."""
    # a path graph long enough that the partial rows exceed 16 MiB at L = 256
    n = 2_400_000
    src = np.arange(n - 1, dtype=np.int64)
    rows = np.concatenate([src, src + 1])
    cols = np.concatenate([src + 1, src])
    order = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    ci = cols[order].astype(np.int32)
    g = api_mod.Graph(ctx, rp, ci)
    need = api_mod.spmm_workspace_size(ctx, g, 1, 256)
    assert need > 16 << 20
    x = torch.zeros((n, 256), dtype=torch.float32, device="cuda")
    out = torch.zeros_like(x)
    with pytest.raises(RuntimeError, match="scratch"):
        api_mod.spmm_noalloc(ctx, g, 1, x, out)
    g.close()
