"""torch.autograd.Function around the unrolled, differentiable PDHG map.

Argument marshalling only: the forward and backward passes run in the HIP
library (pdlp_unroll_*).  Tensors on the GPU are handed over by device
address with the current torch stream (the pdlp_unroll_*_device calls: no
host copies); tensors on the host are handed over as float64 arrays.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Params, Unroll


def _np(t: torch.Tensor) -> np.ndarray:
    return np.ascontiguousarray(t.detach().to("cpu", torch.float64).numpy())


def _f64(t: torch.Tensor) -> torch.Tensor:
    return t.detach().to(torch.float64).contiguous()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


class UnrolledPDHG(torch.autograd.Function):
    """x_K = map(c, lc, uc, val) with the decisions recorded by its own forward
    pass held fixed in the backward pass (see pdlp_unroll_* in include/pdlp.h).
    One forward/backward pair at a time per Unroll object: a later forward
    replaces the recorded decisions, and the backward of an earlier one then
    raises."""

    @staticmethod
    def forward(ctx, c, lc, uc, val, unroll: Unroll, K: int, ckpt: int, params=None):
        if c.is_cuda:
            ts = [_f64(t) for t in (c, lc, uc, val)]
            s = _stream(c.device)
            unroll.set_data_device(*[t.data_ptr() for t in ts], stream=s)
            x = torch.empty(unroll.N, dtype=torch.float64, device=c.device)
            unroll.forward_device(K, ckpt, x.data_ptr(), params, stream=s)
        else:
            unroll.set_data(_np(c), _np(lc), _np(uc), _np(val))
            x = torch.from_numpy(unroll.forward(K, ckpt, params))
        unroll.version = getattr(unroll, "version", 0) + 1
        ctx.unroll, ctx.version, ctx.device = unroll, unroll.version, c.device
        return x

    @staticmethod
    def backward(ctx, gx):
        u = ctx.unroll
        if getattr(u, "version", None) != ctx.version:
            raise RuntimeError("the unrolled map was run forward again before this backward")
        if gx.is_cuda:
            g = _f64(gx)
            out = [torch.empty(k, dtype=torch.float64, device=gx.device)
                   for k in (u.N, u.M, u.M, u.NZ)]
            u.backward_device(g.data_ptr(), *[o.data_ptr() for o in out],
                              stream=_stream(gx.device))
            return (*out, None, None, None, None)
        g = u.backward(_np(gx))
        t = lambda a: torch.from_numpy(a).to(ctx.device)
        return t(g["c"]), t(g["lc"]), t(g["uc"]), t(g["val"]), None, None, None, None


class LPLayer(torch.nn.Module):
    """A batch of LPs with fixed sparsity and variable bounds as a layer:
    forward(c, lc, uc, val) -> x_K (all concatenated over instances)."""

    def __init__(self, lps, K: int = 500, ckpt: int = 25, params: Params | None = None):
        super().__init__()
        self.unroll = Unroll(lps, params)
        self.K, self.ckpt, self.params = int(K), int(ckpt), params

    @classmethod
    def from_tensors(cls, m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, K: int = 500,
                     ckpt: int = 25, params: Params | None = None) -> "LPLayer":
        """The layer of a batch given as CUDA tensors (see Unroll.from_tensors);
        the scalings are those of the data given here."""
        self = cls.__new__(cls)
        torch.nn.Module.__init__(self)
        self.unroll = Unroll.from_tensors(m, n, nnz, row_ptr, col, val, c, lc, uc, lv, uv, params)
        self.K, self.ckpt, self.params = int(K), int(ckpt), params
        return self

    def forward(self, c, lc, uc, val):
        return UnrolledPDHG.apply(c, lc, uc, val, self.unroll, self.K, self.ckpt, self.params)
