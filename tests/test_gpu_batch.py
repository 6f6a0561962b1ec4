"""Batches: many graphs of uneven size in one block-diagonal pass.

Graph g of a batch must give what a run on that graph alone gives with the
same seed: bit for bit where no floating-point sum changes order (NCut and
reduced-modularity projections, GCN, k-means with exact integer centre
sums, integer scores), and to the FP32 feature bar where one does (the
per-graph column sums of the full modularity operator).  Each graph is also
checked against the FP64 oracle stage by stage."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import kmeans as okm
from oracle import projection, scores
from synth import dcsbm

pytestmark = pytest.mark.gpu

COL_TOL = 1e-5
# sizes are ragged on purpose: dense tiles (16 rows) and assignment tiles
# (256 points) straddle graph boundaries
SIZES = [257, 1201, 611, 2003, 90]
SEEDS = [3, 5, 7, 11, 13]
METHOD = dict(proj_dim=64, q=3, layer_dims=[64, 64], k_min=2, k_max=16, k_step=1)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2312_01560_amd import api
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def api_mod():
    from paper_2312_01560_amd import api
    return api


@pytest.fixture(scope="module")
def graphs():
    out = []
    for i, n in enumerate(SIZES):
        k = max(2, int(round(1.6 * n ** 0.35)))
        out.append(dcsbm(n, k, gamma=2.1 + 0.15 * i, d_min=5, d_max=min(n - 1, 150),
                         rho=1.5 + 0.3 * i, seed=200 + i))
    return out


def to_np(t):
    return t.detach().cpu().numpy()


def col_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    nrm = np.linalg.norm(ref, axis=0)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(nrm, 1e-300)


def run_batch(ctx, api_mod, graphs, cfg, seeds):
    hs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, hs)
    out = api_mod.batch_run(ctx, b, cfg, seeds=seeds)
    torch.cuda.synchronize()
    ctx.sync_status()
    res = {k: to_np(v).copy() for k, v in out.items()}
    return b.offsets, res, hs


def run_single(ctx, api_mod, h, cfg):
    out = api_mod.run(ctx, h, cfg)
    torch.cuda.synchronize()
    return {k: to_np(v).copy() for k, v in out.items()}


def test_batch_shape(ctx, api_mod, graphs):
    hs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, hs)
    assert b.G == len(graphs)
    assert b.offsets == [0] + list(np.cumsum(SIZES))
    assert b.nnz == sum(g.nnz for g in graphs)


@pytest.mark.parametrize("op", [0, 2])
def test_batch_equals_single_bit_exact(ctx, api_mod, graphs, op):
    cfg = api_mod.Config(op=op, **METHOD)
    offs, bat, hs = run_batch(ctx, api_mod, graphs, cfg, SEEDS)
    for g, h in enumerate(hs):
        one = run_single(ctx, api_mod, h, api_mod.Config(op=op, seed=SEEDS[g], **METHOD))
        lo, hi = offs[g], offs[g + 1]
        for key in ("Y", "Z", "labels", "labels_all"):
            assert np.array_equal(bat[key][lo:hi], one[key]), (g, key)
        for key in ("k_selected", "mod", "ncut", "picks", "iters"):
            assert np.array_equal(bat[key][g], one[key]), (g, key)


def test_batch_mod_full_matches_single(ctx, api_mod, graphs):
    cfg = api_mod.Config(op=1, **METHOD)
    offs, bat, hs = run_batch(ctx, api_mod, graphs, cfg, SEEDS)
    for g, h in enumerate(hs):
        one = run_single(ctx, api_mod, h, api_mod.Config(op=1, seed=SEEDS[g], **METHOD))
        lo, hi = offs[g], offs[g + 1]
        ref = one["Y"].astype(np.float64)
        assert col_err(bat["Y"][lo:hi], ref).max() < COL_TOL
        assert scores.nmi(bat["labels"][lo:hi], one["labels"]) >= 0.999


def lloyd_step_parity(z32, lab, k, tol=1e-5):
    """The oracle's next Lloyd assignment from the GPU's final labels (FP64
    means of the same FP32 points) keeps every point where the GPU put it,
    up to near-ties.  Lloyd's iteration is not continuous in its inputs:
    rounding-level differences (FP32 against FP64) can send two exact
    implementations to different fixed points, so labels are compared one
    step at a time from the same state."""
    z = z32.astype(np.float64)
    live = [r for r in range(k) if np.any(lab == r)]
    cen = np.stack([z[lab == r].mean(0) for r in live])
    d = okm.sq_distances(z, cen)
    pos = {r: t for t, r in enumerate(live)}
    mine = d[np.arange(len(lab)), [pos[r] for r in lab]]
    assert np.all(mine <= d.min(axis=1) + tol)


@pytest.mark.parametrize("op", [0, 1, 2])
def test_batch_vs_oracle(ctx, api_mod, graphs, op):
    cfg = api_mod.Config(op=op, **METHOD)
    offs, bat, _ = run_batch(ctx, api_mod, graphs, cfg, SEEDS)
    for g, g0 in enumerate(graphs):
        lo, hi = offs[g], offs[g + 1]
        y = projection.project(g0.row_ptr, g0.col_idx, g0.n, op, 64, 3, SEEDS[g])
        z = ogcn.embed(g0.row_ptr, g0.col_idx, g0.n, y, [64, 64], SEEDS[g])
        assert col_err(bat["Y"][lo:hi], y).max() < COL_TOL, g
        assert col_err(bat["Z"][lo:hi], z).max() < COL_TOL, g
        # model selection from the GPU's own FP32 embedding
        z32 = bat["Z"][lo:hi]
        assert np.array_equal(bat["picks"][g], okm.seed_picks(z32, max(cfg.ks), SEEDS[g]))
        lab = bat["labels_all"][lo:hi].astype(np.int64)
        for j, k in enumerate(cfg.ks):
            assert lab[:, j].max() < k
            if bat["iters"][g][j] < cfg.kmeans_max_iter:   # converged: a fixed point
                lloyd_step_parity(z32, lab[:, j], k)
        assert np.mean(bat["iters"][g] < cfg.kmeans_max_iter) > 0.8
        # GPU scores of its own labels are the oracle's scores of those labels
        rmod, rnc = scores.score_candidates(g0.row_ptr, g0.col_idx, lab, cfg.ks)
        assert np.array_equal(bat["mod"][g], rmod)
        assert np.array_equal(bat["ncut"][g], rnc)
        best = scores.select(rmod)
        assert bat["k_selected"][g][0] == cfg.ks[best]
        can, keff = scores.canonical(lab[:, best])
        assert np.array_equal(bat["labels"][lo:hi], can) and bat["k_selected"][g][1] == keff


def test_batch_of_one_is_single(ctx, api_mod, graphs):
    offs, bat, hs = run_batch(ctx, api_mod, graphs[3:4], api_mod.Config(op=1, **METHOD), [9])
    one = run_single(ctx, api_mod, hs[0], api_mod.Config(op=1, seed=9, **METHOD))
    for key in ("Y", "Z", "labels", "labels_all"):
        assert np.array_equal(bat[key], one[key]), key
    for key in ("k_selected", "mod", "ncut", "picks", "iters"):
        assert np.array_equal(bat[key][0], one[key]), key


def test_batch_default_seed_and_repeat(ctx, api_mod, graphs):
    """seeds=None keys every graph with cfg.seed; two runs agree exactly."""
    cfg = api_mod.Config(op=0, seed=4, **METHOD)
    _, a, _ = run_batch(ctx, api_mod, graphs, cfg, None)
    _, b, _ = run_batch(ctx, api_mod, graphs, cfg, [4] * len(graphs))
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_batch_rejects(ctx, api_mod, graphs):
    hs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, hs)
    with pytest.raises(api_mod.RaftError):   # k_max above the smallest graph (90 nodes)
        api_mod.batch_workspace_size(ctx, b, api_mod.Config(op=0, **{**METHOD, "k_max": 91}))
    from synth.dcsbm import edges_to_csr
    rp, ci = edges_to_csr(4, [], [])
    empty = api_mod.Graph(ctx, rp, ci)
    with pytest.raises(api_mod.RaftError):
        api_mod.Batch(ctx, [hs[0], empty])
