"""Batches of graphs (block-diagonal CSR, one launch per stage over all
graphs and candidates, prefix replayed from a HIP graph): every graph's
outputs equal its single-graph run bit for bit, on repeated replays, with and
without the recorded graph; and every graph against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import projection, scores
from synth import dcsbm

pytestmark = pytest.mark.gpu

COL_TOL = 1e-5
FIELDS = ["labels", "k_selected", "mod", "ncut", "labels_all", "picks", "iters", "Y", "Z"]


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


def small_batch():
    sizes = [(90, 3), (2003, 9), (517, 5), (3001, 11), (130, 4), (1200, 7)]
    return [dcsbm(n, k, gamma=2.4, d_min=6, d_max=120, rho=3.0, seed=40 + i)
            for i, (n, k) in enumerate(sizes)]


def to_np(t):
    return t.detach().cpu().numpy()


def single_runs(api_mod, ctx, graphs, cfg, seeds):
    outs = []
    for g0, sd in zip(graphs, seeds):
        g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
        c = api_mod.Config(**{**cfg.__dict__, "seed": sd})
        o = api_mod.run(ctx, g, c)
        torch.cuda.synchronize()
        outs.append({k: to_np(v).copy() for k, v in o.items()})
        g.close()
    return outs


def assert_same(batch_out, ref, tag):
    for g, (bo, r) in enumerate(zip(batch_out, ref)):
        for f in FIELDS:
            got = to_np(bo[f])
            assert np.array_equal(got, r[f]), (tag, g, f)


@pytest.mark.parametrize("op,widths", [(0, (32, [32, 32])), (1, (32, [32, 32])),
                                       (2, (32, [32, 32])), (0, (64, [32, 64]))])
def test_batch_equals_single(ctx, api_mod, op, widths):
    graphs = small_batch()
    cfg = api_mod.Config(op=op, proj_dim=widths[0], q=3, layer_dims=widths[1], k_min=2, k_max=16,
                         normalize_input=widths[0] == 64)
    seeds = [7 + 3 * i for i in range(len(graphs))]
    print(f"batch op={op} G={len(graphs)} n={[g.n for g in graphs]}", flush=True)
    ref = single_runs(api_mod, ctx, graphs, cfg, seeds)
    gs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, gs, cfg, seeds)
    for rep in range(3):                          # replays of the recorded prefix
        out = b.run(want_y=True, want_z=True)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert_same(out, ref, f"replay {rep}")
        # eager work between replays
        torch.zeros(1 << 20, device="cuda").add_(1.0)
        torch.cuda.synchronize()
    b.set_capture(False)
    out = b.run(want_y=True, want_z=True)
    torch.cuda.synchronize()
    assert_same(out, ref, "eager")
    b.close()
    for g in gs:
        g.close()


def test_batch_against_oracle(ctx, api_mod):
    graphs = small_batch()
    cfg = api_mod.Config(op=1, proj_dim=32, q=3, layer_dims=[32, 32], k_min=2, k_max=16)
    gs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, gs, cfg)                # every graph with cfg.seed
    out = b.run(want_y=True, want_z=True)
    torch.cuda.synchronize()
    ctx.sync_status()
    for g0, o in zip(graphs, out):
        y = projection.project(g0.row_ptr, g0.col_idx, g0.n, 1, 32, 3, cfg.seed)
        z = ogcn.embed(g0.row_ptr, g0.col_idx, g0.n, y, [32, 32], cfg.seed)
        yg = to_np(o["Y"]).astype(np.float64)
        zg = to_np(o["Z"]).astype(np.float64)
        ey = np.linalg.norm(yg - y, axis=0) / np.linalg.norm(y, axis=0)
        ez = np.linalg.norm(zg - z, axis=0) / np.linalg.norm(z, axis=0)
        assert ey.max() < COL_TOL and ez.max() < COL_TOL, (g0.n, ey.max(), ez.max())
        lab = to_np(o["labels_all"]).astype(np.int64)
        rmod, rnc = scores.score_candidates(g0.row_ptr, g0.col_idx, lab, cfg.ks)
        assert np.array_equal(to_np(o["mod"]), rmod)
        assert np.array_equal(to_np(o["ncut"]), rnc)
        best = scores.select(rmod)
        can, keff = scores.canonical(lab[:, best])
        ks = to_np(o["k_selected"])
        assert ks[0] == cfg.ks[best] and ks[1] == keff
        assert np.array_equal(to_np(o["labels"]), can)
    b.close()
    for g in gs:
        g.close()


@pytest.fixture(scope="module")
def batch64():
    from synth.workloads import make_batch
    return make_batch(64)


def test_batch64_equals_single(ctx, api_mod, batch64):
    """The batched workload in the benchmark's launch configuration (64 graphs
    of 1k..50k nodes, 0.87 M nodes and 20 M stored entries in one
    block-diagonal CSR, modularity variant, K 2..64): every graph's labels,
    scores, K* and picks equal its single-graph run bit for bit."""
    graphs, method = batch64
    cfg = api_mod.Config(op=1, **method)
    print(f"batch64: N={sum(g.n for g in graphs)} nnz={sum(g.nnz for g in graphs)}", flush=True)
    gs = [api_mod.Graph(ctx, g.row_ptr, g.col_idx) for g in graphs]
    b = api_mod.Batch(ctx, gs, cfg)
    out = b.run()
    torch.cuda.synchronize()
    ctx.sync_status()
    print("batch64: batch run done", flush=True)
    ws = ctx.workspace(max(api_mod.workspace_size(ctx, g, cfg) for g in gs))
    for i, (g, o) in enumerate(zip(gs, out)):
        r = api_mod.run(ctx, g, cfg, ws=ws, want_y=False, want_z=False)
        torch.cuda.synchronize()
        for f in ["labels", "k_selected", "mod", "ncut", "labels_all", "picks", "iters"]:
            assert torch.equal(o[f], r[f]), (i, f)
    b.close()
    for g in gs:
        g.close()


def test_tuner_cache_roundtrip(api_mod, tmp_path):
    """The launch-shape tuner times its candidates on the first run of a new
    workload, writes the choice to the context's cache file, and a new context
    reading that file reuses it without timing; outputs are the same."""
    cache = str(tmp_path / "tune.txt")
    graphs = small_batch()
    cfg = api_mod.Config(op=1, proj_dim=32, q=3, layer_dims=[32, 32], k_min=2, k_max=12)
    outs = []
    for round_ in range(2):
        c = api_mod.Context(0, autotune_cache=cache)
        gs = [api_mod.Graph(c, g.row_ptr, g.col_idx) for g in graphs]
        b = api_mod.Batch(c, gs, cfg)
        o = b.run()
        torch.cuda.synchronize()
        factor, timed = b.tuning()
        if round_ == 0:
            assert len(timed) >= 2 and factor in [f for f, _ in timed]
            first = factor
        else:
            assert timed == [] and factor == first
        outs.append([{k: to_np(v).copy() for k, v in x.items()} for x in o])
        b.close()
        for g in gs:
            g.close()
        c.close()
    with open(cache) as f:
        assert "batch G=6" in f.read()
    for a, b2 in zip(outs[0], outs[1]):
        for k in a:
            assert np.array_equal(a[k], b2[k]), k
