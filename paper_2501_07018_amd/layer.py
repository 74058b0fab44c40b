"""torch.autograd.Function around the unrolled, differentiable PDHG map.

Argument marshalling only: the forward and backward passes run in the HIP
library (pdlp_unroll_forward / pdlp_unroll_backward).  Tensors may live on
any device; they are handed over as float64 host arrays.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Params, Unroll


def _np(t: torch.Tensor) -> np.ndarray:
    return np.ascontiguousarray(t.detach().to("cpu", torch.float64).numpy())


class UnrolledPDHG(torch.autograd.Function):
    """x_K = map(c, lc, uc, val) with the decisions recorded by its own forward
    pass held fixed in the backward pass (see pdlp_unroll_* in include/pdlp.h).
    One forward/backward pair at a time per Unroll object: a later forward
    replaces the recorded decisions, and the backward of an earlier one then
    raises."""

    @staticmethod
    def forward(ctx, c, lc, uc, val, unroll: Unroll, K: int, ckpt: int, params=None):
        unroll.set_data(_np(c), _np(lc), _np(uc), _np(val))
        x = unroll.forward(K, ckpt, params)
        unroll.version = getattr(unroll, "version", 0) + 1
        ctx.unroll, ctx.version, ctx.device = unroll, unroll.version, c.device
        return torch.from_numpy(x).to(c.device)

    @staticmethod
    def backward(ctx, gx):
        u = ctx.unroll
        if getattr(u, "version", None) != ctx.version:
            raise RuntimeError("the unrolled map was run forward again before this backward")
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

    def forward(self, c, lc, uc, val):
        return UnrolledPDHG.apply(c, lc, uc, val, self.unroll, self.K, self.ckpt, self.params)
