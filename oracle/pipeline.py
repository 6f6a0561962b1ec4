"""End-to-end oracle of the hot path: projection -> GCN -> k-means grid ->
scores -> selection (Sec. III: random feature extraction, random embedding
derivation, model selection).  Model selection scans a flat grid of
candidate K; the hierarchical search of Alg. 1 is not part of this path."""
from dataclasses import dataclass, field

import numpy as np

from . import gcn, graph, kmeans, projection, scores


@dataclass
class Config:
    op: int = projection.MOD_FULL
    proj_dim: int = 64
    q: int = 3
    layer_dims: list = field(default_factory=lambda: [64, 64])
    normalize_input: bool = False
    k_min: int = 2
    k_max: int = 30
    k_step: int = 1
    t_max: int = 100
    seed: int = 0

    @property
    def ks(self):
        return kmeans.kgrid(self.k_min, self.k_max, self.k_step)


def run(row_ptr, col_idx, n, cfg: Config, validate=True):
    if validate:
        graph.validate_csr(row_ptr, col_idx, n)
    if graph.two_e(row_ptr) == 0:
        raise graph.CSRError("graph has no edges")
    y = projection.project(row_ptr, col_idx, n, cfg.op, cfg.proj_dim, cfg.q, cfg.seed)
    z = gcn.embed(row_ptr, col_idx, n, y, cfg.layer_dims, cfg.seed, cfg.normalize_input)
    return partition(row_ptr, col_idx, z, cfg) | {"Y": y, "Z": z}


def partition(row_ptr, col_idx, z, cfg: Config):
    ks = cfg.ks
    km = kmeans.multi_k(z, ks, cfg.seed, cfg.t_max)
    mod, nc = scores.score_candidates(row_ptr, col_idx, km["labels"], ks)
    best = scores.select(mod)
    labels, k_eff = scores.canonical(km["labels"][:, best])
    return {"picks": km["picks"], "labels_all": km["labels"], "iters": km["iters"],
            "mod": mod, "ncut": nc, "best": best, "k_star": ks[best],
            "k_eff": k_eff, "labels": labels}
