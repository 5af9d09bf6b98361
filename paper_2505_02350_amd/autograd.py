"""ERBF field as a differentiable torch operation.

``ERBFField.apply(p, lib_ctx, m_dev)`` returns f at every point of the
context's registered levels (eq. 3-9 with the cull of eq. 3-15-1).  Its
backward is the library's vector-Jacobian product: it recomputes the kernel
responses from the parameters instead of keeping any point-kernel pair from
the forward, so the saved state is the parameter tensor alone.
"""

import torch

from . import core


class ERBFField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p: torch.Tensor, lib_ctx: "core.Context", m_dev: torch.Tensor):
        f = lib_ctx.erbf_eval(p.detach(), m_dev)
        ctx.save_for_backward(p, m_dev)
        ctx.lib_ctx = lib_ctx
        return f

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        p, m_dev = ctx.saved_tensors
        g = ctx.lib_ctx.erbf_vjp(p.detach(), m_dev, grad_f.contiguous().float())
        return g, None, None


class ERBFLayer(torch.nn.Module):
    """Holds one packed parameter tensor (``11 * cap_total`` floats, layout
    ``w | c | s | q``) and evaluates the field on a library context."""

    def __init__(self, lib_ctx: "core.Context", p0: torch.Tensor, m_dev: torch.Tensor):
        super().__init__()
        self.lib_ctx = lib_ctx
        self.p = torch.nn.Parameter(p0.detach().clone().float().contiguous())
        self.register_buffer("m_dev", m_dev.detach().clone().to(torch.int32))

    def forward(self) -> torch.Tensor:
        return ERBFField.apply(self.p, self.lib_ctx, self.m_dev)

    def segments(self):
        """Views (w, c, s, q) of the packed parameters, each [k, cap_total]."""
        cap = self.lib_ctx.cap_total
        v = self.p.view(11, cap)
        return v[0:1], v[1:4], v[4:7], v[7:11]
