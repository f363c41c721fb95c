"""Differentiable elasticity solve: u = K(E)^{-1} f with K(E) = sum_e E_e K_e^0.

Forward assembles K(E) on the GPU (element-to-block kernel), builds the aSP-AMG
hierarchy and solves with PCG.  K is symmetric, so the backward pass is one
more solve with the same hierarchy, lam = K^{-1} g_u (the adjoint), followed by
the element-gradient kernel dL/dE_e = -lam_e^T K_e^0 u_e; dL/df = lam.
All numerical work runs in libaspamg.so; this module only wires tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import aspamg


class ElasticModel:
    """Mesh data shared by forward and backward: connectivity, the unit-modulus
    element matrix K_e^0 (shared, 24x24, or per element), the block pattern of
    K with its constrained nodes, and the near-null space for the setup."""

    def __init__(self, n_nodes, conn, Ke0, row_ptr, col, constrained, V0, params=None, device="cuda"):
        self.n_nodes = int(n_nodes)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.V0 = np.ascontiguousarray(V0, dtype=np.float64)
        self.params = params if params is not None else aspamg.default_params()
        self.assembler = aspamg.Assembler(n_nodes, conn, constrained, row_ptr, col, Ke0)
        self.conn = torch.tensor(np.ascontiguousarray(conn, dtype=np.int32), device=device)
        self.Ke0 = torch.tensor(np.ascontiguousarray(Ke0, dtype=np.float64), device=device)
        self.constrained = torch.tensor(np.repeat(np.asarray(constrained, dtype=bool), 3), device=device)

    @classmethod
    def from_problem(cls, p, params=None, device="cuda"):
        return cls(p.n_nodes, p.conn, p.Ke0, p.row_ptr, p.col, p.dirichlet, p.V0, params, device)

    def assemble(self, E):
        return self.assembler(E.detach().contiguous())

    def solver(self, E):
        vals = self.assemble(E)
        torch.cuda.current_stream().synchronize()
        return aspamg.Solver(self.row_ptr, self.col, vals, self.V0, self.params)


class ElasticSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, f, model: ElasticModel):
        S = model.solver(E)
        u = S.solve(f.detach().contiguous())
        ctx.solver = S
        ctx.model = model
        ctx.save_for_backward(u)
        ctx.stats = S.last_stats
        return u

    @staticmethod
    def backward(ctx, g_u):
        (u,) = ctx.saved_tensors
        S, model = ctx.solver, ctx.model
        g = g_u.contiguous().clone()
        g[model.constrained] = 0.0
        lam = S.solve(g)
        grad_E = aspamg.element_gradient(model.conn, model.Ke0, lam, u) if ctx.needs_input_grad[0] else None
        grad_f = lam if ctx.needs_input_grad[1] else None
        S.close()
        return grad_E, grad_f, None


def elastic_solve(E, f, model: ElasticModel):
    """u = K(E)^{-1} f, differentiable in E and f."""
    return ElasticSolve.apply(E, f, model)
