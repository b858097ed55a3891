"""torch.autograd binding of the library's adjoint step (``dg2_adj_*``).

``GaugeDepths.apply(n_cell, Q, adj)`` runs the forward simulation in the
HIP library and returns the gauge depths h[steps, ng] as a float64 tensor;
its backward hands dL/dh to the library's reverse pass and returns dL/dn_cell
and dL/dQ.  Any loss built from h with torch operations (a gauge misfit, a
peak, a weighted sum) differentiates through it; parameter maps such as
per-block Manning values expanded to cells are ordinary torch operations in
front of it.  Argument marshalling only: all arithmetic of the step and of
its adjoint runs in the library's kernels.

The library keeps the checkpoints of the last forward run of an Adjoint
only.  Each node therefore remembers the parameters and the forward count
it ran with; if another forward run on the same Adjoint came in between
(two losses in one graph, a validation run), its backward first repeats its
own forward run, so the gradient always belongs to the node's parameters.
"""
from __future__ import annotations

import numpy as np
import torch

from .dg2 import Adjoint

__all__ = ["GaugeDepths", "DG2Loss", "Adjoint"]


def _rerun_if_stale(adj, run):
    """Repeat a node's forward run if the Adjoint ran another one since."""
    generation, n, q = run
    if adj.generation != generation:
        adj.forward(n, q)


class GaugeDepths(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n_cell: torch.Tensor, Q: torch.Tensor, adj: Adjoint) -> torch.Tensor:
        n = n_cell.detach().to("cpu", torch.float64).numpy()
        q = Q.detach().to("cpu", torch.float64).numpy() if Q is not None else None
        h = adj.forward(n, q)
        ctx.adj = adj
        ctx.run = (adj.generation, n, q)
        ctx.devices = (n_cell.device, n_cell.dtype, None if Q is None else (Q.device, Q.dtype))
        return torch.from_numpy(h).to(n_cell.device)

    @staticmethod
    def backward(ctx, grad_h: torch.Tensor):
        _rerun_if_stale(ctx.adj, ctx.run)
        gn, gq = ctx.adj.backward(grad_h.detach().to("cpu", torch.float64).numpy())
        dev, dt, qinfo = ctx.devices
        gn_t = torch.from_numpy(np.ascontiguousarray(gn)).to(dev, dt)
        gq_t = None if qinfo is None else torch.from_numpy(gq).to(*qinfo)
        return gn_t, gq_t, None


class DG2Loss(torch.autograd.Function):
    """Gauge misfit J = sum over steps and gauges of (h - target)^2 as a
    function of per-block Manning values and the hydrograph samples.

    ``DG2Loss.apply(n_blocks, Q, adj, target, block)``: ``n_blocks`` of shape
    (ny / block, nx / block) is expanded to cells (each block of block x
    block cells shares one value), the library's forward run gives h, and
    the backward run gives dJ/dn per cell, summed back over each block.
    """

    @staticmethod
    def forward(ctx, n_blocks: torch.Tensor, Q: torch.Tensor, adj: Adjoint, target, block: int):
        nb = n_blocks.detach().to("cpu", torch.float64).numpy()
        n_cell = np.kron(nb, np.ones((block, block)))
        q = Q.detach().to("cpu", torch.float64).numpy()
        h = adj.forward(n_cell, q)
        tgt = np.asarray(target.detach().cpu() if torch.is_tensor(target) else target, dtype=np.float64)
        r = h - tgt
        ctx.adj, ctx.block, ctx.r = adj, block, r
        ctx.run = (adj.generation, n_cell, q)
        ctx.meta = (n_blocks.device, n_blocks.dtype, Q.device, Q.dtype, nb.shape)
        return torch.tensor(float((r * r).sum()), dtype=n_blocks.dtype, device=n_blocks.device)

    @staticmethod
    def backward(ctx, grad_J: torch.Tensor):
        g = float(grad_J)
        _rerun_if_stale(ctx.adj, ctx.run)
        gn, gq = ctx.adj.backward(2.0 * g * ctx.r)
        dev, dt, qdev, qdt, (by, bx) = ctx.meta
        b = ctx.block
        gblocks = gn.reshape(by, b, bx, b).sum(axis=(1, 3))
        return (torch.from_numpy(gblocks).to(dev, dt), torch.from_numpy(gq).to(qdev, qdt),
                None, None, None)
