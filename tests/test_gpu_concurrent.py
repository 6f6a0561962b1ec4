"""Contexts driven from several host threads at once, each on its own
stream: independent runs (the NCut and modularity variants of one graph,
and two graphs) overlap on the GPU and every output equals the same run
made alone, bit for bit, over several rounds."""
import threading

import numpy as np
import pytest
import torch

from synth import dcsbm

pytestmark = pytest.mark.gpu

FIELDS = ["labels", "k_selected", "mod", "ncut", "labels_all", "picks", "iters", "Y", "Z"]


@pytest.fixture(scope="module")
def api_mod():
    from paper_2312_01560_amd import api
    return api


def host(outs):
    return {k: outs[k].detach().cpu().numpy() for k in FIELDS if k in outs}


def test_threads_on_own_contexts_equal_serial(api_mod):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    graphs = [dcsbm(3001, 9, gamma=2.2, d_min=5, d_max=200, rho=2.0, seed=11),
              dcsbm(1200, 6, gamma=2.5, d_min=6, d_max=90, rho=2.5, seed=12)]
    # (graph, operator) per job: both variants of one graph, and a second graph
    jobs = [(0, 0), (0, 1), (1, 2)]
    cfgs = [api_mod.Config(op=op, proj_dim=32, q=2, layer_dims=[32, 32], k_min=2, k_max=24,
                           seed=7) for _, op in jobs]
    ctxs = [api_mod.Context(0) for _ in jobs]
    try:
        def run(j):
            c, g0 = ctxs[j], graphs[jobs[j][0]]
            g = api_mod.Graph(c, g0.row_ptr, g0.col_idx)
            out = api_mod.run(c, g, cfgs[j])
            torch.cuda.current_stream().synchronize()
            res = host(out)
            g.close()
            return res

        alone = [run(j) for j in range(len(jobs))]
        streams = [torch.cuda.Stream() for _ in jobs]
        for rnd in range(3):
            got, errors = [None] * len(jobs), []

            def worker(j):
                try:
                    with torch.cuda.stream(streams[j]):
                        got[j] = run(j)
                except BaseException as e:
                    errors.append(e)

            threads = [threading.Thread(target=worker, args=(j,)) for j in range(len(jobs))]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            assert not errors, errors
            for j in range(len(jobs)):
                for k in alone[j]:
                    assert np.array_equal(got[j][k], alone[j][k]), \
                        f"round {rnd}, job {j}: {k} differs from the run alone"
            print(f"round {rnd}: {len(jobs)} concurrent runs equal their runs alone", flush=True)
        for c in ctxs:
            c.sync_status()
    finally:
        torch.cuda.synchronize()
        for c in ctxs:
            c.close()
