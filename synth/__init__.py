"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds no arithmetic of the partitioning method itself: it only
produces graphs (degree-corrected SBM, the paper's generative model, Sec. II
and Sec. IV) and the named workload configurations."""
from .dcsbm import (Graph, bfs_ball, dcsbm, two_cliques, clique_ring, planted_small,  # noqa: F401
                    hub_graph)
from .workloads import WORKLOADS, make_workload, batch_specs  # noqa: F401
