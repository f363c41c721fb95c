"""A mesh above 2,097,152 nodes: the PCG product q = K p then gives each
workgroup several groups of rows so that its p.q partials stay within the
reduction buffer.  Unit cube 128^3 Q1 (129^3 = 2,146,689 nodes, 6.4 M DOF).

  - the first PCG step: u_1 = alpha_0 z_0 with z_0 the V-cycle of f and
    alpha_0 = f.z_0 / z_0.K z_0, recomputed from the library's own operator
    product and V-cycle (checks the fused p.q reduction);
  - 30 iterations: the recursive and recomputed residuals agree."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


def test_pcg_above_two_million_nodes(cuda):
    import torch
    from paper_1902_01715_amd import aspamg
    print("[case cube 128^3, 2,146,689 nodes]", flush=True)
    p = PR.c1_cube(128)
    assert p.n_nodes > 2097152
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(max_it=1, use_graph=0))
    try:
        f = torch.tensor(p.f, device=cuda)
        u1 = S.solve(f, check=False)
        assert S.last_stats["iterations"] == 1
        z0 = S.vcycle(f)
        Kz = S.apply(0, 0, z0)
        alpha_ref = (torch.dot(f, z0) / torch.dot(z0, Kz)).item()
        alpha = (torch.dot(u1, z0) / torch.dot(z0, z0)).item()
        assert abs(alpha - alpha_ref) <= 1e-10 * abs(alpha_ref), (alpha, alpha_ref)
        assert torch.linalg.norm(u1 - alpha_ref * z0).item() <= 1e-10 * torch.linalg.norm(u1).item()
    finally:
        S.close()
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(max_it=30))
    try:
        S.solve(torch.tensor(p.f, device=cuda), check=False)
        st = S.last_stats
        print(f"30 iterations: recursive {st['relres_recursive']:.3e} true {st['relres_true']:.3e}", flush=True)
        assert st["iterations"] == 30 or st["status"] == aspamg.OK
        assert abs(st["relres_recursive"] - st["relres_true"]) <= 1e-8 * max(st["relres_true"], 1e-12) + 1e-13
    finally:
        S.close()
