"""Differentiable solve u = A(theta)^{-1} b over per-element coefficients.

A(theta) = sum_e theta_e R_e^T A_e^(1) R_e (element blocks linear in their
coefficient, the elementwise assembly of Sec. 5.1 of the paper).  The forward
pass builds an LS-AMG-DD hierarchy for A(theta) in the library and solves with
PCG; the backward pass reuses that hierarchy for the adjoint solve
A lambda = ubar (A is symmetric) and contracts the element blocks in the
library: dL/dtheta_e = -sum_k lambda_{k,e}^T A_e^(1) u_{k,e}, dL/db = lambda.
This module only marshals tensors; every solve and contraction runs in liblsdd.
"""
from __future__ import annotations

import numpy as np
import torch

from .lsdd import Hierarchy, Params, elem_bilinear


class ElementSystem:
    """Unit element blocks A_e^(1) and their cover, resident on the device."""

    def __init__(self, prob, params: Params | None = None, device="cuda"):
        self.n = int(prob.n)
        self.elem_ptr = np.ascontiguousarray(prob.elem_ptr, dtype=np.int64)
        self.elem_dofs_host = np.ascontiguousarray(prob.elem_dofs, dtype=np.int32)
        self.elem_dofs = torch.from_numpy(self.elem_dofs_host).to(device)
        self.blocks = torch.from_numpy(np.ascontiguousarray(prob.blocks, dtype=np.float64)).to(device)
        self.node_of_dof = prob.node_of_dof
        self.agg_of_dof = prob.agg_of_dof
        self.params = params or Params.default()
        self.n_elem = len(self.elem_ptr) - 1

    def hierarchy(self, theta: torch.Tensor) -> Hierarchy:
        """Hierarchy of A(theta) (theta: float64 device tensor [n_elem])."""
        return Hierarchy.setup_elements_scaled(self.n, self.elem_ptr, self.elem_dofs_host, self.blocks,
                                               theta.detach().contiguous(), self.node_of_dof, self.agg_of_dof,
                                               self.params)

    def gradient(self, lam: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        """dL/dtheta_e = -sum_k lam_{k,e}^T A_e^(1) u_{k,e} for [n] or [nrhs, n] inputs
        (the sum over right-hand sides and the sign are applied in the library)."""
        return elem_bilinear(self.elem_ptr, self.elem_dofs, self.blocks, lam, u, scale=-1.0)


class ElementSolve(torch.autograd.Function):
    """u = A(theta)^{-1} b; b is [n] or [nrhs, n]."""

    @staticmethod
    def forward(ctx, theta, b, system: ElementSystem):
        h = system.hierarchy(theta)
        u, _ = h.solve(b.detach().contiguous())
        ctx.h, ctx.system = h, system
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, ubar):
        (u,) = ctx.saved_tensors
        h, system = ctx.h, ctx.system
        lam, _ = h.solve(ubar.contiguous())
        g = system.gradient(lam, u)
        h.close()
        ctx.h = None
        return g, lam, None


def solve(theta: torch.Tensor, b: torch.Tensor, system: ElementSystem) -> torch.Tensor:
    """Differentiable u = A(theta)^{-1} b."""
    return ElementSolve.apply(theta, b, system)
