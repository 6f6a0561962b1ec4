"""Named synthetic workloads (graph recipe + method settings).

Each entry gives the DC-SBM recipe and the method settings the workload is run
with.  All are seeded; ``make_workload`` is deterministic.

  small   N=1,000 K=11  gamma 2.5 on [10,100] rho 2.5; L=64 q=3 GCN 64x64;
          candidate K 2..30
  n50k    N=50,000 K=44 gamma 2.5 on [10,300] rho 2.0; L=64 q=3 GCN 64x64;
          candidate K 2..80
  batch64 64 graphs, N log-uniform on [1e3, 5e4], K = round(1.6 N^0.35),
          rho ~ U[1.5,3], gamma ~ U[2.1,2.9], degrees [10,300]; K 2..64
  n1m     N=1,000,000 K=100 gamma 2.3 on [10,1000] rho 2.0; L=128 q=4 GCN
          128x128; candidate K 50..150 step 5
  n200k   N=200,000 K=64 gamma 2.5 on [16,480] rho 2.0; GCN 3x64 (training)
"""
import numpy as np

from .dcsbm import dcsbm

WORKLOADS = {
    "small": dict(graph=dict(n=1000, k=11, alpha=2.0, gamma=2.5, d_min=10, d_max=100, rho=2.5),
                  method=dict(proj_dim=64, q=3, layer_dims=[64, 64], k_min=2, k_max=30, k_step=1)),
    "n50k": dict(graph=dict(n=50000, k=44, alpha=2.0, gamma=2.5, d_min=10, d_max=300, rho=2.0),
                 method=dict(proj_dim=64, q=3, layer_dims=[64, 64], k_min=2, k_max=80, k_step=1)),
    "n1m": dict(graph=dict(n=1000000, k=100, alpha=2.0, gamma=2.3, d_min=10, d_max=1000, rho=2.0),
                method=dict(proj_dim=128, q=4, layer_dims=[128, 128], k_min=50, k_max=150, k_step=5)),
    "n200k": dict(graph=dict(n=200000, k=64, alpha=2.0, gamma=2.5, d_min=16, d_max=480, rho=2.0),
                  method=dict(proj_dim=64, q=3, layer_dims=[64, 64, 64], k_min=2, k_max=64, k_step=1)),
}


def make_workload(name, seed=0):
    w = WORKLOADS[name]
    return dcsbm(seed=seed, **w["graph"]), dict(w["method"])


BATCH_METHOD = dict(proj_dim=64, q=3, layer_dims=[64, 64], k_min=2, k_max=64, k_step=1)


def make_batch(count=64, seed=0):
    """The batched workload: graphs of ``batch_specs`` and its method settings."""
    return [dcsbm(**s) for s in batch_specs(count, seed)], dict(BATCH_METHOD)


def batch_specs(count=64, seed=0, n_lo=1000, n_hi=50000):
    """Per-graph DC-SBM recipes of the batched workload."""
    rng = np.random.default_rng(np.random.SeedSequence([0xB4, int(seed)]))
    specs = []
    for g in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        k = int(round(1.6 * n ** 0.35))
        specs.append(dict(n=n, k=k, alpha=2.0, gamma=float(rng.uniform(2.1, 2.9)),
                          d_min=10, d_max=300, rho=float(rng.uniform(1.5, 3.0)),
                          seed=1000 + g))
    return specs
