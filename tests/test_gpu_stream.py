"""Streaming update on the GPU (raft_stream_*, Sec. III-D): after every batch
of new edges the stream's graph equals the oracle's merged CSR, the rows
recomputed per level equal the oracle's hop balls, and Y and Z equal a fresh
raft_project + raft_embed on the new graph bit for bit (NCut: recomputed on
the balls only; modularity operators: in full); the final embedding against
the FP64 oracle per column; rejected edge sets leave the stream unchanged;
model selection on the stream's graph equals that on a fresh graph."""
import numpy as np
import pytest
import torch

from oracle import streaming
from synth.dcsbm import dcsbm, hub_graph
from synth.workloads import make_workload

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


def new_edges(rp, ci, n, m, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    have = set((rows * n + np.asarray(ci, dtype=np.int64)).tolist())
    out = set()
    while len(out) < m:
        a, b = (int(v) for v in rng.integers(0, n, 2))
        if a == b:
            continue
        a, b = min(a, b), max(a, b)
        if a * n + b in have or (a, b) in out:
            continue
        out.add((a, b))
    e = np.array(sorted(out), dtype=np.int64)
    perm = rng.permutation(len(e))
    return e[perm, 1], e[perm, 0]          # unsorted, larger id first


def fresh(api_mod, ctx, rp, ci, cfg):
    g = api_mod.Graph(ctx, np.asarray(rp, dtype=np.int64), np.asarray(ci, dtype=np.int32))
    y = api_mod.project(ctx, g, cfg)
    z = api_mod.embed(ctx, g, cfg, y)
    torch.cuda.synchronize()
    out = y.cpu().numpy(), z.cpu().numpy()
    g.close()
    return out


def stream_state(st):
    y, z = st.embedding()
    torch.cuda.synchronize()
    return y.cpu().numpy(), z.cpu().numpy()


def col_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


@pytest.mark.parametrize("normalize_input", [False, True])
def test_ncut_stream_equals_fresh(api_mod, ctx, normalize_input):
    g0 = dcsbm(3001, 8, seed=2, d_min=3.0, d_max=30.0)
    n = g0.n
    cfg = api_mod.Config(op=0, proj_dim=32, q=2, layer_dims=[32, 16], k_min=2, k_max=10,
                         normalize_input=normalize_input, seed=5)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    y, z = stream_state(st)
    yf, zf = fresh(api_mod, ctx, g0.row_ptr, g0.col_idx, cfg)
    assert np.array_equal(y, yf) and np.array_equal(z, zf)
    rp, ci = g0.row_ptr.astype(np.int64), g0.col_idx.astype(np.int64)
    radius = cfg.q + len(cfg.layer_dims)
    for batch, m in enumerate([1, 20, 300]):
        s, d = new_edges(rp, ci, n, m, 40 + batch)
        rows = st.add_edges(s, d)
        rp, ci = streaming.add_edges(rp, ci, n, s, d)
        grp, gci = st.graph().csr()
        torch.cuda.synchronize()
        assert np.array_equal(grp.cpu().numpy(), rp) and np.array_equal(gci.cpu().numpy(), ci)
        vprime = np.unique(np.concatenate([s, d]))
        dist = streaming.hop_distance(rp, ci, n, vprime, radius)
        assert rows.tolist() == [int(np.sum(dist <= t)) for t in range(1, radius + 1)]
        print(f"stream batch {batch}: {m} edges, rows per level {rows.tolist()}", flush=True)
        y, z = stream_state(st)
        yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
        assert np.array_equal(y, yf), f"Y differs after batch {batch}"
        assert np.array_equal(z, zf), f"Z differs after batch {batch}"
    assert rows[0] < n                      # the first level really was partial
    ref = streaming.levels(rp, ci, n, 0, cfg.proj_dim, cfg.q, cfg.layer_dims, cfg.seed,
                           normalize_input)
    assert col_err(y, ref["y"][cfg.q]).max() < COL_TOL
    assert col_err(z, ref["h"][-1]).max() < COL_TOL
    st.close()


@pytest.mark.parametrize("proj_dim", [16, 64])
def test_ncut_stream_equals_fresh_hub_rows(api_mod, ctx, proj_dim):
    """Rows of more than 512 entries (summed by a whole wave, their edges
    split over its row groups) recomputed on a stream's partial first level,
    where they sit at other positions of the row list than in a fresh pass:
    Y and Z still equal the fresh run bit for bit."""
    rp0, ci0 = hub_graph(7)
    n = rp0.size - 1
    cfg = api_mod.Config(op=0, proj_dim=proj_dim, q=2, layer_dims=[32], k_min=2, k_max=10,
                         seed=3)
    g = api_mod.Graph(ctx, rp0, ci0)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    rp, ci = rp0.astype(np.int64), ci0.astype(np.int64)
    for batch, m in enumerate([1, 6]):
        s, d = new_edges(rp, ci, n, m, 70 + batch)
        rows = st.add_edges(s, d)
        rp, ci = streaming.add_edges(rp, ci, n, s, d)
        deg = np.diff(rp)
        dist = streaming.hop_distance(rp, ci, n, np.unique(np.concatenate([s, d])), 1)
        assert rows[0] < n and np.sum((dist <= 1) & (deg > 512)) >= 1
        y, z = stream_state(st)
        yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
        assert np.array_equal(y, yf), f"Y differs after batch {batch}"
        assert np.array_equal(z, zf), f"Z differs after batch {batch}"
    st.close()


@pytest.mark.parametrize("op", [1, 2])
def test_modularity_stream_recomputes_all(api_mod, ctx, op):
    g0 = dcsbm(2000, 6, seed=7)
    n = g0.n
    cfg = api_mod.Config(op=op, proj_dim=16, q=3, layer_dims=[16], k_min=2, k_max=8, seed=1)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    rp, ci = g0.row_ptr.astype(np.int64), g0.col_idx.astype(np.int64)
    for batch, m in enumerate([2, 50]):
        s, d = new_edges(rp, ci, n, m, 70 + batch)
        rows = st.add_edges(s, d)
        rp, ci = streaming.add_edges(rp, ci, n, s, d)
        assert rows.tolist() == [n] * 4
        y, z = stream_state(st)
        yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
        assert np.array_equal(y, yf) and np.array_equal(z, zf)
    st.close()


def test_rejected_edges_change_nothing(api_mod, ctx):
    g0 = dcsbm(1000, 5, seed=3)
    n = g0.n
    cfg = api_mod.Config(op=0, proj_dim=16, q=2, layer_dims=[16], k_min=2, k_max=6, seed=2)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    y0, z0 = stream_state(st)
    j = int(g0.col_idx[g0.row_ptr[10]])
    good_s, good_d = new_edges(g0.row_ptr, g0.col_idx, n, 5, 1)
    cases = [
        (np.append(good_s, j), np.append(good_d, 10), -2),   # already present
        (np.array([4]), np.array([4]), -1),                  # self pair
        (np.array([0]), np.array([n]), -1),                  # out of range
        (np.array([1, 2]), np.array([2, 1]), -1),            # the same edge twice
    ]
    for s, d, code in cases:
        with pytest.raises(api_mod.RaftError) as e:
            st.add_edges(s, d)
        assert e.value.status == code
        grp, _ = st.graph().csr()
        y, z = stream_state(st)
        assert int(grp[-1].item()) == g0.nnz
        assert np.array_equal(y, y0) and np.array_equal(z, z0)
    assert st.add_edges(np.zeros(0), np.zeros(0)).tolist() == [0, 0, 0]
    rows = st.add_edges(good_s, good_d)
    assert rows[-1] > 0
    rp, ci = streaming.add_edges(g0.row_ptr, g0.col_idx, n, good_s, good_d)
    y, z = stream_state(st)
    yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
    assert np.array_equal(y, yf) and np.array_equal(z, zf)
    st.close()


def test_partition_on_stream_equals_fresh(api_mod, ctx):
    g0 = dcsbm(2500, 7, seed=11)
    n = g0.n
    cfg = api_mod.Config(op=0, proj_dim=32, q=2, layer_dims=[32], k_min=2, k_max=12, seed=4)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    s, d = new_edges(g0.row_ptr, g0.col_idx, n, 100, 9)
    st.add_edges(s, d)
    rp, ci = streaming.add_edges(g0.row_ptr, g0.col_idx, n, s, d)
    _, z = st.embedding()
    got = api_mod.partition(ctx, st.graph(), cfg, z)
    gf = api_mod.Graph(ctx, rp, ci.astype(np.int32))
    want = api_mod.run(ctx, gf, cfg)
    torch.cuda.synchronize()
    assert np.array_equal(got["labels"].cpu().numpy(), want["labels"].cpu().numpy())
    assert np.array_equal(got["mod"].cpu().numpy(), want["mod"].cpu().numpy())
    gf.close()
    st.close()


def test_n50k_stream(api_mod, ctx):
    g0, method = make_workload("n50k")
    n = g0.n
    cfg = api_mod.Config(op=0, seed=3, **method)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    s, d = new_edges(g0.row_ptr, g0.col_idx, n, 64, 5)
    rows = st.add_edges(s, d)
    print(f"stream n50k: 64 edges, rows per level {rows.tolist()}", flush=True)
    rp, ci = streaming.add_edges(g0.row_ptr, g0.col_idx, n, s, d)
    y, z = stream_state(st)
    yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
    assert np.array_equal(y, yf) and np.array_equal(z, zf)
    st.close()


@pytest.mark.parametrize("layers,width", [([], 32), ([512, 256], 512)])
def test_stream_without_layers_and_wide(api_mod, ctx, layers, width):
    """No GCN layer (the "w/o Emb" form: Z = Y) and Table I widths (512 ->
    512 -> 256): the stream still equals a fresh projection and embedding."""
    g0 = dcsbm(2500, 6, seed=13, d_min=3.0, d_max=30.0)
    n = g0.n
    cfg = api_mod.Config(op=0, proj_dim=width, q=2, layer_dims=layers, k_min=2, k_max=8, seed=6)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    st = api_mod.Stream(ctx, g, cfg)
    g.close()
    rp, ci = g0.row_ptr.astype(np.int64), g0.col_idx.astype(np.int64)
    for batch, m in enumerate([3, 40]):
        s, d = new_edges(rp, ci, n, m, 90 + batch)
        rows = st.add_edges(s, d)
        assert rows.size == cfg.q + len(layers)
        rp, ci = streaming.add_edges(rp, ci, n, s, d)
        y, z = stream_state(st)
        yf, zf = fresh(api_mod, ctx, rp, ci, cfg)
        assert np.array_equal(y, yf) and np.array_equal(z, zf)
    st.close()
