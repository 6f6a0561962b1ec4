"""Host-only checks of the batch planner (no GPU): for the batched workload's
graph sizes and for edge shapes (one graph, tiny graphs next to large ones,
wide layers, no GCN layers, input normalisation), every array each graph's
kernels index lies inside that graph's part of the workspace, the control
block or the packed features, and every launch table covers its graph."""
import numpy as np
import pytest

from synth import batch_specs


def _api():
    from paper_2312_01560_amd import api
    return api


def _cfg(**kw):
    api = _api()
    base = dict(op=api.X_MOD_FULL, proj_dim=64, q=3, layer_dims=[64, 64], k_min=2, k_max=64)
    base.update(kw)
    return api.Config(**base)


def test_batched_workload_layout():
    specs = batch_specs(64)
    ns = [s["n"] for s in specs]
    # stored entries of the order the generator gives (mean degree ~ 25)
    nnzs = [25 * n for n in ns]
    st, msg = _api().batch_plan_check(ns, nnzs, _cfg())
    assert st == 0, msg


@pytest.mark.parametrize("kw", [
    dict(),
    dict(op=0, proj_dim=128, layer_dims=[128, 128], k_min=50, k_max=150, k_step=5),
    dict(layer_dims=[], proj_dim=32),
    dict(normalize_input=True, layer_dims=[64, 32, 128]),
    dict(op=2, k_min=1, k_max=12),
    dict(proj_dim=256, layer_dims=[16, 256]),
])
def test_edge_shapes(kw):
    rng = np.random.default_rng(3)
    ns = [151, 2, 70001, 1000, 64, 65, 3001] + list(rng.integers(200, 20000, 9))
    cfg = _cfg(**kw)
    ns = [max(n, cfg.k_max) for n in ns]
    nnzs = [2 * n for n in ns]
    st, msg = _api().batch_plan_check(ns, nnzs, cfg)
    assert st == 0, msg


def test_single_graph_batch():
    st, msg = _api().batch_plan_check([50000], [1203370], _cfg(k_max=80))
    assert st == 0, msg


def test_rejects_k_max_above_n():
    st, _ = _api().batch_plan_check([100, 10], [400, 40], _cfg(k_max=30))
    assert st != 0


def test_rejects_int32_overflow():
    st, _ = _api().batch_plan_check([2_000_000] * 2, [1_200_000_000] * 2, _cfg())
    assert st != 0
