"""Trainable-weight mode of the random GCN: autograd Functions over the
library's hand-written adjoints (raft_gcn_forward/backward,
raft_modloss_forward/backward) and Adam (raft_adam_step).

The loss relaxes the matrix form of modularity (Eq. 4): -tr(S^T B S)/2e with
S the row softmax of the last (linear) layer's logits.  The paper itself never
trains (Sec. III-B); the random weights are step 0 of this model.
"""
import ctypes

import torch

from .api import _ptr, _stream


def _dims_arr(dims):
    return (ctypes.c_int32 * len(dims))(*dims)


def _ptr_arr(tensors):
    return (ctypes.c_void_p * max(1, len(tensors)))(*[t.data_ptr() for t in tensors])


class Trainer:
    """Holds the graph, the workspace and the per-layer buffers."""

    def __init__(self, ctx, graph, dims):
        self.ctx, self.g, self.dims = ctx, graph, list(dims)
        self.nl = len(dims) - 1
        n = ctypes.c_size_t()
        ctx.check(ctx.lib.raft_train_workspace_size(ctx.h, graph.h, self.nl, _dims_arr(dims),
                                                    dims[-1], ctypes.byref(n)))
        self.ws = ctx.workspace(n.value)

    def forward(self, H0, Ws):
        n = self.g.n
        saved = [self.ctx.empty((n, self.dims[k + 1]), torch.float32) for k in range(self.nl - 1)]
        U = self.ctx.empty((n, self.dims[-1]), torch.float32)
        self.ctx.check(self.ctx.lib.raft_gcn_forward(
            self.ctx.h, self.g.h, self.nl, _dims_arr(self.dims), _ptr(H0), _ptr_arr(Ws),
            _ptr_arr(saved), _ptr(U), _ptr(self.ws), self.ws.numel(), _stream()))
        return U, saved

    def backward(self, H0, Ws, saved, G_U, want_h0=False):
        GW = [torch.empty_like(w) for w in Ws]
        GH0 = torch.empty_like(H0) if want_h0 else None
        self.ctx.check(self.ctx.lib.raft_gcn_backward(
            self.ctx.h, self.g.h, self.nl, _dims_arr(self.dims), _ptr(H0), _ptr_arr(Ws),
            _ptr_arr(saved), _ptr(G_U.contiguous()), _ptr_arr(GW), _ptr(GH0), _ptr(self.ws),
            self.ws.numel(), _stream()))
        return GW, GH0

    def modloss_forward(self, U):
        K = U.shape[1]
        S = torch.empty_like(U)
        loss = self.ctx.empty((1,), torch.float64)
        self.ctx.check(self.ctx.lib.raft_modloss_forward(
            self.ctx.h, self.g.h, _ptr(U.contiguous()), K, _ptr(S), _ptr(loss), _ptr(self.ws),
            self.ws.numel(), _stream()))
        return S, loss

    def modloss_backward(self, S, scale=None):
        G = torch.empty_like(S)
        self.ctx.check(self.ctx.lib.raft_modloss_backward(
            self.ctx.h, self.g.h, _ptr(S), S.shape[1], _ptr(scale), _ptr(G), _ptr(self.ws),
            self.ws.numel(), _stream()))
        return G

    def adam(self, w, m, v, g, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
        self.ctx.check(self.ctx.lib.raft_adam_step(
            self.ctx.h, _ptr(w), _ptr(m), _ptr(v), _ptr(g), w.numel(), lr, b1, b2, eps, step,
            _stream()))


class RaftGCN(torch.autograd.Function):
    """U = GCN(H0; W_1..W_n): hidden layers tanh + row normalisation, last
    layer linear.  Only the layer inputs are kept; backward recomputes."""

    @staticmethod
    def forward(ctx, trainer, H0, *Ws):
        H0 = H0.contiguous()
        Ws = [w.contiguous() for w in Ws]
        U, saved = trainer.forward(H0, Ws)
        ctx.trainer = trainer
        ctx.save_for_backward(H0, *Ws, *saved)
        ctx.nl = len(Ws)
        return U

    @staticmethod
    def backward(ctx, G_U):
        t = ctx.saved_tensors
        nl = ctx.nl
        H0, Ws, saved = t[0], list(t[1:1 + nl]), list(t[1 + nl:])
        GW, GH0 = ctx.trainer.backward(H0, Ws, saved, G_U, want_h0=ctx.needs_input_grad[1])
        return (None, GH0, *GW)


class RaftModLoss(torch.autograd.Function):
    """loss = -tr(S^T B S)/2e with S = softmax_rows(U)."""

    @staticmethod
    def forward(ctx, trainer, U):
        S, loss = trainer.modloss_forward(U)
        ctx.trainer = trainer
        ctx.save_for_backward(S)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (S,) = ctx.saved_tensors
        scale = g.reshape(1).to(torch.float32).contiguous()
        return None, ctx.trainer.modloss_backward(S, scale)
