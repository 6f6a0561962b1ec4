"""Python binding of the HIP library: device memory and streams come from
torch; every computation is a call into libraftgp.so."""
import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import RaftConfig, RaftOutputs, X_GCN, X_MOD_FULL, X_MOD_REDUCED, X_NCUT  # noqa: F401

STREAM_THETA = 0x10
STREAM_W_BASE = 0x10


class RaftError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"raftgp error {status}: {message}")
        self.status = status


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Config:
    """Method settings (mirror of raft_config)."""
    op: int = X_MOD_FULL
    proj_dim: int = 64
    q: int = 3
    layer_dims: list = field(default_factory=lambda: [64, 64])
    normalize_input: bool = False
    k_min: int = 2
    k_max: int = 30
    k_step: int = 1
    kmeans_max_iter: int = 100
    check_every: int = 4
    kmeans_prune: int = 0   # 0 where it pays (mean K >= 64), 1 always, 2 never
    seed: int = 0

    @property
    def ks(self):
        return list(range(self.k_min, self.k_max + 1, self.k_step))

    @property
    def embed_dim(self):
        return self.layer_dims[-1] if self.layer_dims else self.proj_dim

    def to_c(self):
        c = RaftConfig()
        c.abi_version = _lib.ABI_VERSION
        c.op = self.op
        c.proj_dim = self.proj_dim
        c.q = self.q
        c.n_layers = len(self.layer_dims)
        for i, v in enumerate(self.layer_dims):
            c.layer_dims[i] = v
        c.normalize_input = int(bool(self.normalize_input))
        c.k_min, c.k_max, c.k_step = self.k_min, self.k_max, self.k_step
        c.kmeans_max_iter = self.kmeans_max_iter
        c.check_every = self.check_every
        c.kmeans_prune = int(self.kmeans_prune)
        c.seed = self.seed
        return c


class Context:
    def __init__(self, device=0, autotune_cache=None):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        cache = autotune_cache.encode() if autotune_cache else None
        st = self.lib.raft_ctx_create(device, cache, ctypes.byref(h))
        if st != 0:
            raise RaftError(st, "raft_ctx_create failed")
        self.h = h
        self.torch_device = torch.device("cuda", device)

    def check(self, st):
        if st != 0:
            buf = ctypes.create_string_buffer(1024)
            self.lib.raft_last_error(self.h, buf, 1024)
            raise RaftError(st, buf.value.decode(errors="replace"))

    def sync_status(self):
        self.check(self.lib.raft_sync_status(self.h, _stream()))

    def close(self):
        if self.h:
            self.lib.raft_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.torch_device)

    def workspace(self, nbytes):
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.torch_device)
        assert ws.data_ptr() % 256 == 0
        return ws


class Graph:
    """Device CSR owned by the library (raft_graph)."""

    def __init__(self, ctx, row_ptr, col_idx, n=None):
        """row_ptr: int32 or int64 offsets (int64 ones are checked and
        narrowed by the library); col_idx: int32.  Host (numpy) or device
        (torch) arrays."""
        self.ctx = ctx
        if isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda:
            wide = row_ptr.dtype == torch.int64
            rp = row_ptr.contiguous() if wide else row_ptr.to(torch.int32).contiguous()
            ci = col_idx.to(torch.int32).contiguous()
            on_dev = 1
            rp_p, ci_p = _ptr(rp), _ptr(ci)
            nnz = ci.numel()
            keep = (rp, ci)
        else:
            wide = np.asarray(row_ptr).dtype == np.int64
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64 if wide else np.int32)
            ci = np.ascontiguousarray(col_idx, dtype=np.int32)
            on_dev = 0
            rp_p = rp.ctypes.data_as(ctypes.c_void_p)
            ci_p = ci.ctypes.data_as(ctypes.c_void_p)
            nnz = ci.size
            keep = (rp, ci)
        self.n = int(len(rp) - 1) if n is None else int(n)
        self.nnz = int(nnz)
        h = ctypes.c_void_p()
        st = ctx.lib.raft_graph_create(ctx.h, rp_p, int(wide), ci_p, self.n, self.nnz, on_dev,
                                       _stream(), ctypes.byref(h))
        del keep
        ctx.check(st)
        self.h = h

    @classmethod
    def _from_handle(cls, ctx, h):
        g = cls.__new__(cls)
        g.ctx, g.h = ctx, h
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        ctx.check(ctx.lib.raft_graph_size(h, ctypes.byref(n), ctypes.byref(nnz)))
        g.n, g.nnz = int(n.value), int(nnz.value)
        return g

    def degrees(self):
        out = self.ctx.empty((self.n,), torch.int32)
        self.ctx.check(self.ctx.lib.raft_graph_degrees(self.h, _ptr(out), _stream()))
        return out

    def csr(self):
        """The library's CSR as device tensors (row_ptr int32 [N + 1],
        col_idx int32 [nnz])."""
        rp = self.ctx.empty((self.n + 1,), torch.int32)
        ci = self.ctx.empty((max(self.nnz, 1),), torch.int32)
        self.ctx.check(self.ctx.lib.raft_graph_csr(self.h, _ptr(rp), _ptr(ci), _stream()))
        return rp, ci[: self.nnz]

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owned", True):
                self.ctx.lib.raft_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(ctx, g, cfg):
    c = cfg.to_c()
    n = ctypes.c_size_t()
    ctx.check(ctx.lib.raft_workspace_size(ctx.h, g.h, ctypes.byref(c), ctypes.byref(n)))
    return n.value


def gaussian(ctx, seed, stream_id, rows, cols, sigma):
    out = ctx.empty((rows, cols), torch.float32)
    ctx.check(ctx.lib.raft_gaussian(ctx.h, seed, stream_id, rows, cols, float(sigma), _ptr(out),
                                    _stream()))
    return out


def spmm_workspace_size(ctx, g, op, L):
    n = ctypes.c_size_t()
    ctx.check(ctx.lib.raft_spmm_workspace_size(ctx.h, g.h, op, L, ctypes.byref(n)))
    return n.value


def spmm(ctx, g, op, Y, out=None, ws=None):
    Y = Y.contiguous()
    L = Y.shape[1]
    out = ctx.empty((g.n, L), torch.float32) if out is None else out
    need = spmm_workspace_size(ctx, g, op, L)
    if need and (ws is None or ws.numel() < need):
        ws = ctx.workspace(need)
    ctx.check(ctx.lib.raft_spmm(ctx.h, g.h, op, L, Y.data_ptr(), out.data_ptr(),
                                ws.data_ptr() if need else None, ws.numel() if need else 0,
                                _stream()))
    return out


def spmm_merge(ctx, g, op, Y, out=None, ws=None):
    """raft_spmm_merge: the merge-path split of the same product."""
    Y = Y.contiguous()
    L = Y.shape[1]
    out = ctx.empty((g.n, L), torch.float32) if out is None else out
    need = ctypes.c_size_t()
    ctx.check(ctx.lib.raft_spmm_merge_workspace_size(ctx.h, g.h, op, L, ctypes.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = ctx.workspace(need.value)
    ctx.check(ctx.lib.raft_spmm_merge(ctx.h, g.h, op, L, Y.data_ptr(), out.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream()))
    return out


def spmm_noalloc(ctx, g, op, Y, out):
    """raft_spmm_noalloc: the caller passes the output; the library allocates
    nothing (MOD_FULL's partials live in its fixed per-GPU scratch)."""
    ctx.check(ctx.lib.raft_spmm_noalloc(ctx.h, g.h, op, Y.shape[1], Y.data_ptr(),
                                        out.data_ptr(), _stream()))
    return out


def _ws_for(ctx, g, cfg, ws):
    need = workspace_size(ctx, g, cfg)
    if ws is None or ws.numel() < need:
        ws = ctx.workspace(need)
    return ws


def project(ctx, g, cfg, ws=None, out=None):
    ws = _ws_for(ctx, g, cfg, ws)
    out = ctx.empty((g.n, cfg.proj_dim), torch.float32) if out is None else out
    c = cfg.to_c()
    ctx.check(ctx.lib.raft_project(ctx.h, g.h, ctypes.byref(c), _ptr(ws), ws.numel(), _ptr(out),
                                   _stream()))
    return out


def gcn_layer(ctx, g, H, W, linear=False, want_p=False):
    H = H.contiguous()
    W = W.contiguous()
    lin, lout = W.shape
    out = ctx.empty((g.n, lout), torch.float32)
    P = ctx.empty((g.n, lin), torch.float32)
    ctx.check(ctx.lib.raft_gcn_layer(ctx.h, g.h, lin, lout, _ptr(H), _ptr(W), int(linear),
                                     _ptr(out), _ptr(P), ctypes.c_void_p(0), 0, _stream()))
    return (out, P) if want_p else out


def embed(ctx, g, cfg, Y, ws=None, out=None):
    ws = _ws_for(ctx, g, cfg, ws)
    out = ctx.empty((g.n, cfg.embed_dim), torch.float32) if out is None else out
    c = cfg.to_c()
    ctx.check(ctx.lib.raft_embed(ctx.h, g.h, ctypes.byref(c), _ptr(Y.contiguous()), _ptr(ws),
                                 ws.numel(), _ptr(out), _stream()))
    return out


def _outputs(ctx, g, cfg, want_y=False, want_z=False, want_centres=False):
    kc = len(cfg.ks)
    o = {
        "labels": ctx.empty((g.n,), torch.int32),
        "k_selected": ctx.empty((3,), torch.int32),
        "mod": ctx.empty((kc,), torch.float64),
        "ncut": ctx.empty((kc,), torch.float64),
        "labels_all": ctx.empty((g.n, kc), torch.uint8),
        "picks": ctx.empty((max(cfg.ks),), torch.int32),
        "iters": ctx.empty((kc,), torch.int32),
    }
    if want_y:
        o["Y"] = ctx.empty((g.n, cfg.proj_dim), torch.float32)
    if want_z:
        o["Z"] = ctx.empty((g.n, cfg.embed_dim), torch.float32)
    if want_centres:
        o["centres"] = ctx.empty((sum(cfg.ks), cfg.embed_dim), torch.float32)
    s = RaftOutputs()
    for name, _ in RaftOutputs._fields_:
        t = o.get(name)
        setattr(s, name, t.data_ptr() if t is not None else None)
    return o, s


def partition(ctx, g, cfg, Z, ws=None, want_centres=False):
    ws = _ws_for(ctx, g, cfg, ws)
    o, s = _outputs(ctx, g, cfg, want_centres=want_centres)
    c = cfg.to_c()
    ctx.check(ctx.lib.raft_partition(ctx.h, g.h, ctypes.byref(c), _ptr(Z.contiguous()),
                                     _ptr(ws), ws.numel(), ctypes.byref(s), _stream()))
    return o


def run(ctx, g, cfg, ws=None, want_y=True, want_z=True, outputs=None, want_centres=False):
    """A1-A7 on one graph; returns a dict of device tensors."""
    ws = _ws_for(ctx, g, cfg, ws)
    if outputs is None:
        outputs = _outputs(ctx, g, cfg, want_y, want_z, want_centres)
    o, s = outputs
    c = cfg.to_c()
    ctx.check(ctx.lib.raft_run(ctx.h, g.h, ctypes.byref(c), _ptr(ws), ws.numel(), ctypes.byref(s),
                               _stream()))
    return o


class Batch:
    """Many graphs through the whole path at once (raft_batch): one
    block-diagonal CSR on the device, one launch per stage over all graphs
    and candidates.  Graph g uses seeds[g] (cfg.seed when None)."""

    def __init__(self, ctx, graphs, cfg, seeds=None):
        self.ctx = ctx
        self.cfg = cfg
        self.graphs = list(graphs)
        G = len(self.graphs)
        hs = (ctypes.c_void_p * G)(*[g.h.value for g in self.graphs])
        sd = None
        if seeds is not None:
            sd = (ctypes.c_uint64 * G)(*[int(v) for v in seeds])
        self.seeds = list(seeds) if seeds is not None else [cfg.seed] * G
        c = cfg.to_c()
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.raft_batch_create(ctx.h, G, hs, sd, ctypes.byref(c), ctypes.byref(h)))
        self.h = h
        need = ctypes.c_size_t()
        ctx.check(ctx.lib.raft_batch_workspace_size(ctx.h, self.h, ctypes.byref(need)))
        self.ws_bytes = need.value
        self.ws = None

    def set_capture(self, enable):
        self.ctx.check(self.ctx.lib.raft_batch_set_capture(self.h, int(bool(enable))))

    def outputs(self, want_y=False, want_z=False):
        return [_outputs(self.ctx, g, self.cfg, want_y, want_z) for g in self.graphs]

    def run(self, outputs=None, want_y=False, want_z=False):
        """Returns one dict of device tensors per graph (as api.run)."""
        if self.ws is None:
            self.ws = self.ctx.workspace(self.ws_bytes)
        if outputs is None:
            outputs = self.outputs(want_y, want_z)
        arr = (RaftOutputs * len(outputs))(*[s for _, s in outputs])
        self.ctx.check(self.ctx.lib.raft_batch_run(self.ctx.h, self.h, _ptr(self.ws),
                                                   self.ws.numel(), arr, _stream()))
        return [o for o, _ in outputs]

    def stage_times(self):
        arr = (ctypes.c_double * 3)()
        self.ctx.check(self.ctx.lib.raft_batch_stage_times(self.h, arr))
        return list(arr)

    def tuning(self):
        """(chosen factor, [(candidate, ms), ...]) of the launch-shape tuner."""
        f = ctypes.c_int32()
        cnt = ctypes.c_int32()
        arr = (ctypes.c_double * 32)()
        self.ctx.check(self.ctx.lib.raft_batch_tuning(self.h, ctypes.byref(f), arr, 16,
                                                      ctypes.byref(cnt)))
        return f.value, [(int(arr[2 * i]), arr[2 * i + 1]) for i in range(cnt.value)]

    def close(self):
        if self.h:
            self.ctx.lib.raft_batch_destroy(self.h)
            self.h = None


def batch_plan_check(ns, nnzs, cfg, num_cu=256):
    """Host-only check of the batch planner (no GPU): (status, message)."""
    lib = _lib.load()
    G = len(ns)
    n_arr = (ctypes.c_int32 * G)(*[int(v) for v in ns])
    e_arr = (ctypes.c_int64 * G)(*[int(v) for v in nnzs])
    c = cfg.to_c()
    msg = ctypes.create_string_buffer(512)
    st = lib.raft_batch_plan_check(G, n_arr, e_arr, ctypes.byref(c), num_cu, msg, 512)
    return st, msg.value.decode(errors="replace")


def hier_partition(ctx, g, Z, eps=5, t_max=100, seed=0, trace_depth=0):
    """Alg. 1 on the embedding Z (device [N x d]).  Returns dict(labels
    (device int32 [N]), k (blocks), tree (list of dicts, tree node order),
    trace (device int32 [trace_depth x N] or None))."""
    Z = Z.contiguous()
    d = Z.shape[1]
    need = ctypes.c_size_t()
    ctx.check(ctx.lib.raft_hier_workspace_size(ctx.h, g.h, d, ctypes.byref(need)))
    ws = ctx.workspace(need.value)
    labels = ctx.empty((g.n,), torch.int32)
    trace = ctx.empty((trace_depth, g.n), torch.int32) if trace_depth > 0 else None
    cfg = _lib.RaftHierConfig(eps, t_max, seed)
    cap = 2 * g.n + 1
    nodes = (_lib.RaftHierNode * cap)()
    nb = ctypes.c_int32()
    nt = ctypes.c_int32()
    ctx.check(ctx.lib.raft_hier_partition(
        ctx.h, g.h, _ptr(Z), d, ctypes.byref(cfg), _ptr(ws), ws.numel(), _ptr(labels),
        ctypes.byref(nb), nodes, cap, ctypes.byref(nt), _ptr(trace) if trace is not None else None,
        trace_depth, _stream()))
    tree = [{"depth": x.depth, "size": x.size, "parent": x.parent, "child": list(x.child),
             "block": x.block, "kmeans_iters": x.kmeans_iters, "sizes": list(x.sizes),
             "m1": x.m1, "m2": x.m2} for x in nodes[:nt.value]]
    return {"labels": labels, "k": nb.value, "tree": tree, "trace": trace}


def score(ctx, g, labels_all, ks):
    labels_all = labels_all.to(torch.uint8).contiguous()
    kc = len(ks)
    mod = ctx.empty((kc,), torch.float64)
    nc = ctx.empty((kc,), torch.float64)
    ks_arr = (ctypes.c_int32 * kc)(*ks)
    need = ctypes.c_size_t()
    ctx.check(ctx.lib.raft_score_workspace_size(ctx.h, g.h, kc, ks_arr, ctypes.byref(need)))
    ws = ctx.workspace(need.value)
    ctx.check(ctx.lib.raft_score(ctx.h, g.h, _ptr(labels_all), kc, ks_arr, _ptr(mod), _ptr(nc),
                                 _ptr(ws), ws.numel(), _stream()))
    return mod, nc


def confusion(ctx, a, b, ka=None, kb=None):
    """Contingency counts [ka x kb] (int64, device) of two device labelings."""
    a = a.to(torch.int32).contiguous()
    b = b.to(torch.int32).contiguous()
    ka = int(a.max().item()) + 1 if ka is None else int(ka)
    kb = int(b.max().item()) + 1 if kb is None else int(kb)
    out = ctx.empty((ka, kb), torch.int64)
    ctx.check(ctx.lib.raft_confusion(ctx.h, _ptr(a), _ptr(b), a.numel(), ka, kb, _ptr(out),
                                     _stream()))
    return out


def nmi(ctx, a, b):
    """NMI of two device labelings: counts on the device, finish on the host."""
    counts = confusion(ctx, a, b)
    host = np.ascontiguousarray(counts.cpu().numpy(), dtype=np.int64)
    ctx.sync_status()
    val = ctypes.c_double()
    st = ctx.lib.raft_nmi_from_counts(host.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      host.shape[0], host.shape[1], ctypes.byref(val))
    ctx.check(st)
    return val.value


def stage_times(ctx):
    arr = (ctypes.c_double * 5)()
    ctx.check(ctx.lib.raft_get_stage_times(ctx.h, arr))
    return list(arr)


def profile_enable(ctx, mask):
    ctx.check(ctx.lib.raft_profile_enable(ctx.h, mask))


def profile_read(ctx):
    """{class: (ms, launches)} accumulated since the last read."""
    ms = (ctypes.c_double * _lib.PROF_CLASSES)()
    n = (ctypes.c_int64 * _lib.PROF_CLASSES)()
    ctx.check(ctx.lib.raft_profile_read(ctx.h, ms, n))
    names = ["spmm", "dense", "race", "assign", "update", "score"]
    return {names[k]: (ms[k], n[k]) for k in range(_lib.PROF_CLASSES)}


def sbm_sample(ctx, theta, blocks, omega, seed):
    """A graph sampled from the degree-corrected SBM by the fast jump sampler
    (Sec. IV, Alg. 2) on the device: theta [n] FP64, blocks [n] int in
    0..k-1, omega [k x k] FP64 symmetric (host arrays).  Returns a Graph."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    blocks = np.ascontiguousarray(blocks, dtype=np.int32)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    if omega.ndim != 2 or omega.shape[0] != omega.shape[1]:
        raise ValueError("omega must be k x k")
    if theta.shape != blocks.shape or theta.ndim != 1:
        raise ValueError("theta and blocks must be vectors of one length")
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.raft_sbm_sample(ctx.h, theta.size, omega.shape[0],
                                      theta.ctypes.data_as(ctypes.c_void_p),
                                      blocks.ctypes.data_as(ctypes.c_void_p),
                                      omega.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_uint64(int(seed)), _stream(), ctypes.byref(h)))
    return Graph._from_handle(ctx, h)


class Stream:
    """A graph and every level of its embedding, updated as edges arrive
    (Sec. III-D): under NCut each level is recomputed on the hop ball of the
    new edges' endpoints only; under the modularity operators in full."""

    def __init__(self, ctx, g, cfg):
        self.ctx, self.cfg, self.n = ctx, cfg, g.n
        c = cfg.to_c()
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.raft_stream_create(ctx.h, g.h, ctypes.byref(c), _stream(),
                                             ctypes.byref(h)))
        self.h = h

    @property
    def levels(self):
        return self.cfg.q + len(self.cfg.layer_dims)

    def add_edges(self, src, dst):
        """Adds the undirected edges (src[e], dst[e]); returns the rows
        recomputed at each level (numpy int64, q + layers entries)."""
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        rows = np.zeros(self.levels, dtype=np.int64)
        self.ctx.check(self.ctx.lib.raft_stream_add_edges(
            self.h, src.ctypes.data_as(ctypes.c_void_p), dst.ctypes.data_as(ctypes.c_void_p),
            src.size, _stream(), rows.ctypes.data_as(ctypes.c_void_p)))
        return rows

    def graph(self):
        """The current graph (owned by the stream; valid until the next
        add_edges or close)."""
        h = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.raft_stream_graph(self.h, ctypes.byref(h)))
        g = Graph._from_handle(self.ctx, h)
        g._owned = False
        return g

    def embedding(self):
        """(Y [N x L], Z [N x d]) device copies of the current levels."""
        y = self.ctx.empty((self.n, self.cfg.proj_dim), torch.float32)
        z = self.ctx.empty((self.n, self.cfg.embed_dim), torch.float32)
        self.ctx.check(self.ctx.lib.raft_stream_embedding(self.h, _ptr(y), _ptr(z), _stream()))
        return y, z

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.raft_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
