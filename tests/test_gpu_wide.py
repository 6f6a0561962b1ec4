"""The paper's layer configurations (Table I: projection widths up to 4096,
GCN widths down to the embedding) and the "w/o Emb" ablation (Table IV: the
projection itself as the embedding): SpMM at wide L per column against the
FP64 oracle, single wide GCN layers, and whole runs against the oracle."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import graph as ograph
from oracle import pipeline, projection, scores
from synth import dcsbm

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


@pytest.fixture(scope="module")
def g5k():
    # the N = 5E3 row of Table I: K = 19, degrees about 5..164
    return dcsbm(5000, 19, gamma=2.5, d_min=5, d_max=160, rho=3.0, seed=51)


@pytest.mark.parametrize("op", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [512, 4096])
def test_wide_spmm(ctx, api_mod, g5k, op, L):
    g = api_mod.Graph(ctx, g5k.row_ptr, g5k.col_idx)
    x = np.random.default_rng(L + op).standard_normal((g5k.n, L)).astype(np.float32)
    got = api_mod.spmm(ctx, g, op, torch.from_numpy(x).cuda()).cpu().numpy()
    rp, ci, n = g5k.row_ptr, g5k.col_idx, g5k.n
    x64 = x.astype(np.float64)
    if op == 0:
        ref = projection.ncut_operator(rp, ci, n) @ x64
    elif op == 1:
        a = ograph.adjacency(rp, ci, n)
        d = ograph.degrees(rp).astype(float)
        ref = projection.apply_modularity(a, d, float(ograph.two_e(rp)), x64)
    elif op == 2:
        ref = projection.reduced_modularity_operator(rp, ci, n) @ x64
    else:
        ref = ogcn.gcn_operator(rp, ci, n) @ x64
    assert col_err(got, ref).max() < COL_TOL
    g.close()


@pytest.mark.parametrize("lin,lout", [(4096, 2048), (1024, 512), (512, 256), (256, 512),
                                      (2048, 128)])
def test_wide_gcn_layer(ctx, api_mod, g5k, lin, lout):
    g = api_mod.Graph(ctx, g5k.row_ptr, g5k.col_idx)
    rng = np.random.default_rng(lin + lout)
    h = rng.standard_normal((g5k.n, lin)).astype(np.float32)
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    w = (rng.standard_normal((lin, lout)) / np.sqrt(lin)).astype(np.float32)
    got = api_mod.gcn_layer(ctx, g, torch.from_numpy(h).cuda(), torch.from_numpy(w).cuda())
    p = ogcn.gcn_operator(g5k.row_ptr, g5k.col_idx, g5k.n) @ h.astype(np.float64)
    z = np.tanh(p @ w.astype(np.float64))
    z /= np.maximum(np.linalg.norm(z, axis=1, keepdims=True), 1e-12)
    assert col_err(got.cpu().numpy(), z).max() < COL_TOL
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_table1_config_5k(ctx, api_mod, g5k, op):
    """Table I at N = 5E3: L = 1024, GCN widths 512, 256, 128 (d = 128)."""
    m = dict(proj_dim=1024, q=3, layer_dims=[512, 256, 128], k_min=2, k_max=30)
    g = api_mod.Graph(ctx, g5k.row_ptr, g5k.col_idx)
    cfg = api_mod.Config(op=op, **m)
    out = api_mod.run(ctx, g, cfg)
    torch.cuda.synchronize()
    ctx.sync_status()
    y = projection.project(g5k.row_ptr, g5k.col_idx, g5k.n, op, 1024, 3, 0)
    z = ogcn.embed(g5k.row_ptr, g5k.col_idx, g5k.n, y, [512, 256, 128], 0)
    assert col_err(out["Y"].cpu().numpy(), y).max() < COL_TOL
    assert col_err(out["Z"].cpu().numpy(), z).max() < COL_TOL
    lab = out["labels_all"].cpu().numpy().astype(np.int64)
    rmod, _ = scores.score_candidates(g5k.row_ptr, g5k.col_idx, lab, cfg.ks)
    assert np.array_equal(out["mod"].cpu().numpy(), rmod)
    assert scores.nmi(out["labels"].cpu().numpy(), g5k.planted) > 0.9
    g.close()


def test_table1_config_10k_embedding(ctx, api_mod):
    """Table I at N = 1E4: L = 4096, GCN widths 2048, 1024, 512, 256."""
    g0 = dcsbm(10000, 25, gamma=2.5, d_min=6, d_max=180, rho=3.0, seed=52)
    m = dict(proj_dim=4096, q=1, layer_dims=[2048, 1024, 512, 256])
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    cfg = api_mod.Config(op=0, **m)
    y = api_mod.project(ctx, g, cfg)
    z = api_mod.embed(ctx, g, cfg, y)
    torch.cuda.synchronize()
    ctx.sync_status()
    yr = projection.project(g0.row_ptr, g0.col_idx, g0.n, 0, 4096, 1, 0)
    assert col_err(y.cpu().numpy(), yr).max() < COL_TOL
    zr = ogcn.embed(g0.row_ptr, g0.col_idx, g0.n, yr, m["layer_dims"], 0)
    assert col_err(z.cpu().numpy(), zr).max() < COL_TOL
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_without_embedding_ablation(ctx, api_mod, small_graph, op):
    """Table IV (ii) "w/o Emb": no GCN layer, the projection Y is the
    embedding; Y = Z and the selection against the oracle."""
    g0, m = small_graph
    m = dict(m, layer_dims=[])
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    cfg = api_mod.Config(op=op, **m)
    out = api_mod.run(ctx, g, cfg)
    torch.cuda.synchronize()
    ctx.sync_status()
    assert torch.equal(out["Y"], out["Z"])
    ref = pipeline.run(g0.row_ptr, g0.col_idx, g0.n, pipeline.Config(op=op, **m))
    assert col_err(out["Z"].cpu().numpy(), ref["Z"]).max() < COL_TOL
    lab = out["labels_all"].cpu().numpy().astype(np.int64)
    rmod, _ = scores.score_candidates(g0.row_ptr, g0.col_idx, lab, cfg.ks)
    assert np.array_equal(out["mod"].cpu().numpy(), rmod)
    sel = pipeline.partition(g0.row_ptr, g0.col_idx, out["Z"].cpu().numpy().astype(np.float64),
                             pipeline.Config(op=op, **m))
    assert scores.nmi(out["labels"].cpu().numpy(), sel["labels"]) >= 0.999
    g.close()
