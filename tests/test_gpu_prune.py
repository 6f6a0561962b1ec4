"""Bound-pruned Lloyd assignment (Hamerly's bounds, from the third
assignment on): runs that skip the points whose bounds prove their label
give the labels, k-means++ picks, iteration counts, centres, scores and the
selected K of runs that score every point in every iteration, bit for bit:
across embedding widths 32/64/128, the three operators, grids that include
K = 1, ragged sizes, short T_max and several poll periods, and from given
embeddings at very large and very small scales (the score error bound
scales with the norms)."""
import numpy as np
import pytest
import torch

from synth import dcsbm, make_workload

pytestmark = pytest.mark.gpu

KEYS = ("labels_all", "iters", "picks", "centres", "mod", "ncut", "k_selected", "labels")


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


@pytest.fixture(scope="module")
def ragged():
    return dcsbm(3001, 9, gamma=2.2, d_min=5, d_max=400, rho=2.0, seed=11)


def to_host(o):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def run_both(api_mod, ctx, g, **cfg):
    out = {}
    for dense in (False, True):
        c = api_mod.Config(kmeans_prune=2 if dense else 1, **cfg)
        out[dense] = to_host(api_mod.run(ctx, g, c, want_centres=True))
    ctx.sync_status()
    return out


def assert_same(out, keys=KEYS):
    for key in keys:
        a, b = out[False][key], out[True][key]
        assert a.shape == b.shape and np.array_equal(a, b), key


@pytest.mark.parametrize("op", [0, 1, 2])
@pytest.mark.parametrize("dims", [[64, 64], [32], [64, 128]])
def test_pruned_equals_dense(api_mod, ctx, ragged, op, dims):
    g = api_mod.Graph(ctx, ragged.row_ptr, ragged.col_idx)
    out = run_both(api_mod, ctx, g, op=op, proj_dim=64, q=3, layer_dims=dims,
                   k_min=1, k_max=40, k_step=1, seed=5)
    assert_same(out)
    print(f"op {op} dims {dims}: iterations {int(out[False]['iters'].sum())}", flush=True)
    g.close()


@pytest.mark.parametrize("t_max,every", [(3, 1), (4, 2), (9, 7), (100, 1)])
def test_pruned_short_runs_and_polls(api_mod, ctx, ragged, t_max, every):
    g = api_mod.Graph(ctx, ragged.row_ptr, ragged.col_idx)
    out = run_both(api_mod, ctx, g, op=0, proj_dim=64, q=2, layer_dims=[64],
                   k_min=2, k_max=60, k_step=3, kmeans_max_iter=t_max, check_every=every,
                   seed=1)
    assert_same(out)
    assert out[False]["iters"].max() <= t_max
    g.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_pruned_equals_dense_n50k(api_mod, ctx, variant):
    graph, m = make_workload("n50k")
    g = api_mod.Graph(ctx, graph.row_ptr, graph.col_idx)
    out = run_both(api_mod, ctx, g, op=variant, **m)
    assert_same(out)
    print(f"n50k op {variant}: K* {out[False]['k_selected'][0]}, "
          f"iterations {int(out[False]['iters'].sum())}", flush=True)
    g.close()


def gaussian_mixture(n, d, k, scale, seed):
    rng = np.random.default_rng(seed)
    centres = rng.normal(size=(k, d)) * 3.0
    lab = rng.integers(0, k, n)
    z = centres[lab] + rng.normal(size=(n, d))
    return (z * scale).astype(np.float32)


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e4])
@pytest.mark.parametrize("d", [64, 128])
def test_pruned_partition_from_embedding(api_mod, ctx, ragged, scale, d):
    """Partition of a given Z (a Gaussian mixture, not row-normalised) at
    three scales: pruned == dense, bit for bit."""
    g = api_mod.Graph(ctx, ragged.row_ptr, ragged.col_idx)
    z = torch.from_numpy(gaussian_mixture(ragged.n, d, 12, scale, seed=d)).cuda()
    out = {}
    for dense in (False, True):
        cfg = api_mod.Config(kmeans_prune=2 if dense else 1, op=1, proj_dim=d, layer_dims=[d], k_min=2,
                             k_max=50, k_step=1, seed=3)
        out[dense] = to_host(api_mod.partition(ctx, g, cfg, z, want_centres=True))
    ctx.sync_status()
    assert_same(out, ("labels_all", "iters", "picks", "centres", "mod", "ncut", "k_selected"))
    g.close()


def test_pruned_large_point_set(api_mod, ctx):
    """140,001 clustered points at d = 128 on a ring graph, K = 2..62 step 4
    (the assignment's group-major block order, several candidate groups)."""
    n, d = 140001, 128
    rp = (2 * np.arange(n + 1)).astype(np.int32)
    nb = np.stack([(np.arange(n) - 1) % n, (np.arange(n) + 1) % n], axis=1)
    ci = np.sort(nb, axis=1).reshape(-1).astype(np.int32)
    rng = np.random.default_rng(5)
    dirs = rng.standard_normal((40, d))
    z = dirs[rng.integers(0, 40, n)] + 0.5 * rng.standard_normal((n, d))
    z = (z / np.linalg.norm(z, axis=1, keepdims=True)).astype(np.float32)
    g = api_mod.Graph(ctx, rp, ci)
    zt = torch.from_numpy(z).cuda()
    out = {}
    for dense in (False, True):
        cfg = api_mod.Config(kmeans_prune=2 if dense else 1, op=0, proj_dim=d, layer_dims=[d], k_min=2,
                             k_max=62, k_step=4, kmeans_max_iter=300)
        out[dense] = to_host(api_mod.partition(ctx, g, cfg, zt, want_centres=True))
    ctx.sync_status()
    assert_same(out, ("labels_all", "iters", "picks", "centres", "mod", "ncut", "k_selected"))
    g.close()


def test_automatic_mode_prunes_large_k(api_mod, ctx, ragged):
    """The default mode prunes grids with a mean K of 64 or more (here d =
    128, K = 64..128 step 8) and gives the results of a run that never
    prunes; an out-of-range mode is rejected."""
    g = api_mod.Graph(ctx, ragged.row_ptr, ragged.col_idx)
    out = {}
    for dense in (False, True):
        c = api_mod.Config(kmeans_prune=2 if dense else 0, op=1, proj_dim=128, q=2,
                           layer_dims=[128], k_min=64, k_max=128, k_step=8, seed=2)
        out[dense] = to_host(api_mod.run(ctx, g, c, want_centres=True))
    ctx.sync_status()
    assert_same(out)
    with pytest.raises(RuntimeError):
        api_mod.run(ctx, g, api_mod.Config(kmeans_prune=3, k_min=2, k_max=10))
    g.close()


def test_pruned_tiny_and_isolated(api_mod, ctx):
    """Graphs smaller than one range and one wave (two K5 cliques and a
    bridge; a ring with isolated nodes, whose embedding rows are zero):
    pruned == dense, bit for bit."""
    from synth import two_cliques
    g0 = two_cliques(5)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    out = run_both(api_mod, ctx, g, op=1, proj_dim=32, q=2, layer_dims=[32], k_min=1, k_max=6,
                   seed=4)
    assert_same(out)
    g.close()
    n = 300
    ring = np.arange(200)
    src = np.concatenate([ring, ring])
    dst = np.concatenate([(ring + 1) % 200, (ring + 7) % 200])
    from synth.dcsbm import edges_to_csr
    rp, ci = edges_to_csr(n, src, dst)          # nodes 200..299 isolated
    g = api_mod.Graph(ctx, rp, ci)
    out = run_both(api_mod, ctx, g, op=0, proj_dim=64, q=2, layer_dims=[64], k_min=2, k_max=40,
                   k_step=2, seed=6)
    assert_same(out)
    g.close()
