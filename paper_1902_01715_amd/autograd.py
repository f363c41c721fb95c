"""Differentiable elasticity solve: u = K(E)^{-1} f with K(E) = sum_e E_e K_e^0.

Forward assembles K(E) on the GPU (element-to-block kernel), builds the aSP-AMG
hierarchy and solves with PCG.  K is symmetric, so the backward pass is one
more solve with the same hierarchy, lam = K^{-1} g_u (the adjoint), followed by
the element-gradient kernel dL/dE_e = -lam_e^T K_e^0 u_e; dL/df = lam.
Constrained DOFs are decoupled identity rows of K (u_c = f_c, no coupling to
the free DOFs), so dL/df_c = dL/du_c there and the element gradient sees u with
its constrained entries zeroed (K(E) holds no free-constrained couplings).
A solve that does not reach its tolerance raises (strict models, the default)
or warns.  All numerical work runs in libaspamg.so; this module only wires
tensors.
"""
from __future__ import annotations

import warnings

import numpy as np
import torch

from . import aspamg


class ElasticModel:
    """Mesh data shared by forward and backward: connectivity, the unit-modulus
    element matrix K_e^0 (shared, 24x24, or per element), the block pattern of
    K with its constrained nodes, and the near-null space for the setup."""

    def __init__(self, n_nodes, conn, Ke0, row_ptr, col, constrained, V0, params=None, device="cuda", strict=True):
        self.strict = bool(strict)
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

    def checked_solve(self, S, rhs, what):
        x = S.solve(rhs)
        st = S.last_stats
        if st["status"] != aspamg.OK:
            msg = (f"{what} solve did not converge: status {st['status']}, {st['iterations']} iterations, "
                   f"relres {st['relres_recursive']:.2e} (recomputed {st['relres_true']:.2e})")
            if self.strict:
                S.close()
                raise RuntimeError(msg)
            warnings.warn(msg, RuntimeWarning, stacklevel=3)
        return x


class ElasticSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, f, model: ElasticModel):
        S = model.solver(E)
        u = model.checked_solve(S, f.detach().contiguous(), "forward")
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
        lam = model.checked_solve(S, g, "adjoint")
        grad_E = None
        if ctx.needs_input_grad[0]:
            uf = u.clone()
            uf[model.constrained] = 0.0
            grad_E = aspamg.element_gradient(model.conn, model.Ke0, lam, uf)
        grad_f = None
        if ctx.needs_input_grad[1]:
            grad_f = lam.clone()
            grad_f[model.constrained] = g_u[model.constrained]
        S.close()
        return grad_E, grad_f, None


def elastic_solve(E, f, model: ElasticModel):
    """u = K(E)^{-1} f, differentiable in E and f."""
    return ElasticSolve.apply(E, f, model)
