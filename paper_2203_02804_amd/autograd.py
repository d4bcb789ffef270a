"""torch.autograd.Function around the batched pricer: prices forward, delta and vega backward.

The backward pass is the adjoint of the tensor-train contraction computed by the library
(node moments of the frozen cores combined with the derivative of the characteristic
function), so no second TT-cross is run. The derivative is that of the fixed-grid
quadrature: the grid (L, alpha per term and coordinate) is frozen at the forward inputs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Pricer, plan


def _options(S0, sigma, base):
    S0 = S0.detach().cpu().double().numpy()
    sigma = sigma.detach().cpu().double().numpy()
    out = []
    for i in range(S0.shape[0]):
        o = dict(base[i])
        o["S0"] = S0[i].tolist()
        o["sigma"] = sigma[i].tolist()
        out.append(o)
    return out


class TTPrice(torch.autograd.Function):
    """prices = TTPrice.apply(S0[n, d], sigma[n, d], pricer, options, grids).

    options: list of n option dicts (their S0 / sigma are replaced by the tensors' rows);
    grids: list of n grid dicts with explicit L / alpha (see frozen_grids)."""

    @staticmethod
    def forward(ctx, S0, sigma, pricer: Pricer, options, grids):
        opts = _options(S0, sigma, options)
        prices, delta, vega, status = pricer.price_batch(opts, grids, greeks=True)
        dev = S0.device
        ctx.save_for_backward(torch.tensor(np.stack(delta), dtype=torch.float64, device=dev),
                              torch.tensor(np.stack(vega), dtype=torch.float64, device=dev))
        return torch.tensor(prices, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, grad):
        delta, vega = ctx.saved_tensors
        g = grad.to(torch.float64)[:, None]
        return g * delta, g * vega, None, None, None


def frozen_grids(options, grid):
    """Per-option grid dicts whose L / alpha are the arrays the pricer chooses at the given
    parameters, so that derivatives are taken at a fixed quadrature grid."""
    out = []
    for o in options:
        L, A = plan(o, grid)
        out.append(dict(grid, L=L, alpha=A))
    return out
