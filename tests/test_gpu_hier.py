"""Hierarchical model selection on the GPU (Sec. III-C, Alg. 1, local
modularity Eq. 7) against the FP64 oracle: given the GPU's K = 2 splits, the
oracle's Alg. 1 visits the same sets, computes the same LMod values bit for
bit and takes the same decisions (the same tree and the same block labels);
the GPU's K = 2 splits agree with the oracle's KMeans on the same sets; and
the planted cliques of a clique ring are recovered."""
import numpy as np
import pytest
import torch

from oracle import gcn as ogcn
from oracle import hierarchical as ohier
from oracle import projection, scores
from synth import clique_ring, make_workload

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


TRACE = 96


def replay_with_gpu_splits(g0, out, seed=0, eps=5):
    """The oracle's Alg. 1 with each KMeans split replaced by the GPU's."""
    tr = out["trace"].cpu().numpy()
    tree = out["tree"]

    def split(nodes, depth):
        assert depth < TRACE
        v = tr[depth, nodes]
        t = v // 2
        assert np.all(t == t[0]) and np.sum(tr[depth] // 2 == t[0]) == nodes.size
        assert tree[t[0]]["kmeans_iters"] > 0
        return (v % 2).astype(np.int64)
    return ohier.partition(g0.row_ptr, g0.col_idx, None, seed=seed, eps=eps, splitter=split)


def same_float(a, b):
    if a is None:
        return np.isnan(b)
    return a == b


def check_tree(out, ref):
    tr = out["trace"].cpu().numpy()
    tree = out["tree"]
    assert len(ref["tree"]) == len(tree)
    for depth, nodes, decision, m1, m2, sizes in ref["tree"]:
        t = tr[depth, nodes[0]] // 2
        node = tree[t]
        assert node["depth"] == depth and node["size"] == nodes.size
        assert same_float(m1, node["m1"]), (depth, nodes.size, m1, node["m1"])
        assert same_float(m2, node["m2"]), (depth, nodes.size, m2, node["m2"])
        assert (decision == "block") == (node["child"][0] < 0)
        if sizes is not None:
            assert tuple(sizes) == tuple(node["sizes"])
    assert np.array_equal(out["labels"].cpu().numpy(), ref["labels"])
    assert out["k"] == ref["k"]


def gpu_embedding(api_mod, ctx, g0, m, op):
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    cfg = api_mod.Config(op=op, **m)
    z = api_mod.embed(ctx, g, cfg, api_mod.project(ctx, g, cfg))
    torch.cuda.synchronize()
    return g, z


@pytest.mark.parametrize("op", [0, 1])
def test_tree_equals_oracle_given_splits(ctx, api_mod, small_graph, op):
    g0, m = small_graph
    g, z = gpu_embedding(api_mod, ctx, g0, m, op)
    out = api_mod.hier_partition(ctx, g, z, trace_depth=TRACE)
    print(f"hier op={op}: {out['k']} blocks, {len(out['tree'])} tree nodes", flush=True)
    ref = replay_with_gpu_splits(g0, out)
    check_tree(out, ref)
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_splits_match_oracle_kmeans(ctx, api_mod, small_graph, op):
    """Each KMeans split of the GPU against the oracle's KMeans (race and
    Lloyd in FP64) on the same set and FP32 points; and the whole partition
    against the oracle's Alg. 1 on the same points."""
    g0, m = small_graph
    g, z = gpu_embedding(api_mod, ctx, g0, m, op)
    out = api_mod.hier_partition(ctx, g, z, trace_depth=TRACE)
    tr = out["trace"].cpu().numpy()
    z64 = z.cpu().numpy().astype(np.float64)
    agree = total = 0
    for t, node in enumerate(out["tree"]):
        if node["kmeans_iters"] == 0:
            continue
        depth = node["depth"]
        nodes = np.flatnonzero(tr[depth] // 2 == t)
        mine = tr[depth, nodes] % 2
        ref = ohier.split_two(z64, nodes, 0, depth)
        agree += int(np.sum(mine == ref))
        total += nodes.size
    assert total > 0 and agree >= 0.999 * total, (agree, total)
    full = ohier.partition(g0.row_ptr, g0.col_idx, z64, seed=0)
    assert scores.nmi(out["labels"].cpu().numpy(), full["labels"]) >= 0.999
    g.close()


def test_clique_ring_recovered(ctx, api_mod):
    g0 = clique_ring(6, 12)
    y = projection.project(g0.row_ptr, g0.col_idx, g0.n, 1, 32, 3, 0)
    z = ogcn.embed(g0.row_ptr, g0.col_idx, g0.n, y, [32, 32], 0).astype(np.float32)
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    out = api_mod.hier_partition(ctx, g, torch.from_numpy(z).cuda(), trace_depth=TRACE)
    assert out["k"] == 6
    assert scores.nmi(out["labels"].cpu().numpy(), g0.planted) == 1.0
    ref = ohier.partition(g0.row_ptr, g0.col_idx, z.astype(np.float64), seed=0)
    assert np.array_equal(out["labels"].cpu().numpy(), ref["labels"])
    check_tree(out, replay_with_gpu_splits(g0, out))
    g.close()


def test_small_graph_is_one_block(ctx, api_mod):
    from synth import two_cliques
    g0 = two_cliques(5)                     # 10 nodes <= 2 eps + 1
    g = api_mod.Graph(ctx, g0.row_ptr, g0.col_idx)
    z = torch.randn(g0.n, 32, device="cuda")
    out = api_mod.hier_partition(ctx, g, z, trace_depth=4)
    assert out["k"] == 1 and out["labels"].cpu().numpy().tolist() == [0] * 10
    assert out["tree"][0]["kmeans_iters"] == 0
    g.close()


@pytest.mark.parametrize("eps", [0, 2, 20])
def test_eps_values(ctx, api_mod, small_graph, eps):
    g0, m = small_graph
    g, z = gpu_embedding(api_mod, ctx, g0, m, 1)
    out = api_mod.hier_partition(ctx, g, z, eps=eps, trace_depth=TRACE)
    ref = replay_with_gpu_splits(g0, out, eps=eps)
    check_tree(out, ref)
    g.close()


def test_n50k_tree_equals_oracle_given_splits(ctx, api_mod):
    """At the benchmark's size (N = 50,000, GPU embedding): the tree and
    labels against the oracle's Alg. 1 replayed with the GPU's splits."""
    g0, m = make_workload("n50k")
    g, z = gpu_embedding(api_mod, ctx, g0, m, 1)
    out = api_mod.hier_partition(ctx, g, z, trace_depth=TRACE)
    print(f"hier n50k: {out['k']} blocks, depth {max(t['depth'] for t in out['tree'])}",
          flush=True)
    check_tree(out, replay_with_gpu_splits(g0, out))
    g.close()
