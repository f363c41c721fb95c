"""The adjoint-sensitivity workload at full size (SIMP cube 48^3, 352,947 DOF,
110,592 elements): the compliance gradient from the adjoint solve and the
element-gradient kernel against central finite differences (h = 1e-6, energy
form of the compliance) on the 20 sampled elements of the generator, the Euler
identity sum_e rho_e dC/drho_e = -3 C, and the oracle's element-gradient
formula applied to the GPU solution."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


def test_c5_gradient_full_size(cuda, oracle_lib):
    import torch
    from paper_1902_01715_amd import aspamg
    from paper_1902_01715_amd.autograd import ElasticModel, elastic_solve
    print("[case c5 full size]", flush=True)
    p = PR.c5_simp()
    assert len(p.extra["fd_elems"]) == 20
    model = ElasticModel.from_problem(p, aspamg.default_params(rtol=1e-12))
    rho = torch.tensor(p.extra["rho"], device="cuda", requires_grad=True)
    f = torch.tensor(p.f, device="cuda")
    u = elastic_solve(rho ** 3, f, model)
    C = torch.dot(f, u)
    C.backward()
    g = rho.grad.cpu().numpy()
    Cv = C.item()
    un = u.detach().cpu().numpy()
    g_o = 3 * p.extra["rho"] ** 2 * oracle_lib.element_gradient(p.conn, p.Ke0, un, un)
    assert np.abs(g - g_o).max() <= 1e-9 * np.abs(g_o).max()
    assert abs((p.extra["rho"] * g).sum() + 3 * Cv) <= 1e-8 * Cv
    h = 1e-6
    worst = 0.0
    for e in p.extra["fd_elems"]:
        cs = []
        for s in (+1, -1):
            r = p.extra["rho"].copy()
            r[e] += s * h
            S = model.solver(torch.tensor(r ** 3, device="cuda"))
            up = S.solve(f)
            Ku = S.apply(0, 0, up)
            cs.append((2 * torch.dot(f, up) - torch.dot(up, Ku)).item())
            S.close()
        fd = (cs[0] - cs[1]) / (2 * h)
        worst = max(worst, abs(fd - g[e]) / abs(g[e]))
        assert abs(fd - g[e]) <= 1e-3 * abs(g[e]) + 1e-9 * Cv / g.size, (e, fd, g[e])
    print(f"largest relative FD difference over 20 elements: {worst:.2e}")
