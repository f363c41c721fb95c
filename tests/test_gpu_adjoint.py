"""Adjoint sensitivity on the GPU: element-to-block assembly, the adjoint solve
and the element-gradient kernel, against the CPU oracle, central finite
differences (energy form of the compliance) and the Euler identity
sum_e rho_e dC/drho_e = -3 C of SIMP (K(t rho) = t^3 K(rho) on the free DOFs)."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def simp(cuda):
    from paper_1902_01715_amd import aspamg
    from paper_1902_01715_amd.autograd import ElasticModel
    print("[case simp 10^3]", flush=True)
    p = PR.c5_simp(10, seed=5, n_fd=8)
    model = ElasticModel.from_problem(p, aspamg.default_params(rtol=1e-12))
    return p, model


def test_gpu_assembly_matches_generator(simp):
    import torch
    p, model = simp
    E = torch.tensor(p.E, device="cuda")
    vals = model.assemble(E).cpu().numpy()
    scale = np.abs(p.vals).max()
    assert np.abs(vals - p.vals).max() <= 1e-13 * scale


def test_element_gradient_kernel_matches_oracle(simp, oracle_lib):
    import torch
    from paper_1902_01715_amd import aspamg
    p, model = simp
    rng = np.random.default_rng(0)
    lam = rng.standard_normal(p.n_dof)
    u = rng.standard_normal(p.n_dof)
    g_ref = oracle_lib.element_gradient(p.conn, p.Ke0, lam, u)
    g = aspamg.element_gradient(model.conn, model.Ke0, torch.tensor(lam, device="cuda"),
                                torch.tensor(u, device="cuda")).cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-12 * np.abs(g_ref).max()
    # per-element matrices (stride 576) give the same result
    Ke = np.broadcast_to(p.Ke0, (p.conn.shape[0], 24, 24)).copy()
    g2 = aspamg.element_gradient(model.conn, torch.tensor(Ke, device="cuda"), torch.tensor(lam, device="cuda"),
                                 torch.tensor(u, device="cuda")).cpu().numpy()
    assert np.abs(g2 - g_ref).max() <= 1e-12 * np.abs(g_ref).max()


def test_compliance_gradient(simp, oracle_lib):
    import torch
    from paper_1902_01715_amd.autograd import elastic_solve
    p, model = simp
    rho = torch.tensor(p.extra["rho"], device="cuda", requires_grad=True)
    f = torch.tensor(p.f, device="cuda")
    u = elastic_solve(rho ** 3, f, model)
    C = torch.dot(f, u)
    C.backward()
    g = rho.grad.cpu().numpy()
    Cv = C.item()
    # oracle gradient with the oracle's own solve
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    u_o, st = H.pcg(p.f, 1e-12, 1000)
    g_o = 3 * p.extra["rho"] ** 2 * oracle_lib.element_gradient(p.conn, p.Ke0, u_o, u_o)
    assert np.abs(g - g_o).max() <= 1e-7 * np.abs(g_o).max()
    # Euler identity
    assert abs((p.extra["rho"] * g).sum() + 3 * Cv) <= 1e-8 * Cv
    # central differences in energy form on sampled elements
    h = 1e-6
    for e in p.extra["fd_elems"]:
        cs = []
        for s in (+1, -1):
            r = p.extra["rho"].copy()
            r[e] += s * h
            E = torch.tensor(r ** 3, device="cuda")
            S = model.solver(E)
            up = S.solve(f)
            Ku = S.apply(0, 0, up)
            cs.append((2 * torch.dot(f, up) - torch.dot(up, Ku)).item())
            S.close()
        fd = (cs[0] - cs[1]) / (2 * h)
        assert abs(fd - g[e]) <= 1e-3 * abs(g[e]) + 1e-9 * Cv / g.size, (e, fd, g[e])


def test_load_gradient_and_clamped_loads(cuda):
    """L = w . u with loads also on clamped nodes (there u_c = f_c: decoupled
    identity rows).  dL/df against exact central differences (L is linear in
    f), dL/dE against central differences on sampled elements, both through
    the autograd function; the clamped loads must not leak into dL/dE."""
    import torch
    from paper_1902_01715_amd import aspamg
    from paper_1902_01715_amd.autograd import ElasticModel, elastic_solve
    print("[case clamped loads simp 6^3]", flush=True)
    p = PR.c5_simp(6, seed=7, n_fd=6)
    model = ElasticModel.from_problem(p, aspamg.default_params(rtol=1e-12))
    rng = np.random.default_rng(1)
    f0 = p.f.copy()
    cdof = np.repeat(p.dirichlet, 3)
    f0[cdof] = rng.standard_normal(cdof.sum())
    w = torch.tensor(rng.standard_normal(p.n_dof), device="cuda")
    E0 = p.extra["rho"] ** 3

    def loss(E, f):
        u = elastic_solve(torch.tensor(E, device="cuda"), torch.tensor(f, device="cuda"), model)
        return torch.dot(w, u).item()

    E = torch.tensor(E0, device="cuda", requires_grad=True)
    f = torch.tensor(f0, device="cuda", requires_grad=True)
    L = torch.dot(w, elastic_solve(E, f, model))
    L.backward()
    gE, gf = E.grad.cpu().numpy(), f.grad.cpu().numpy()
    # constrained DOFs: u_c = f_c, so dL/df_c = w_c exactly
    assert np.abs(gf[cdof] - w.cpu().numpy()[cdof]).max() == 0.0
    free = np.flatnonzero(~cdof)
    for i in list(rng.choice(free, 4, replace=False)) + list(np.flatnonzero(cdof)[:2]):
        fp, fm = f0.copy(), f0.copy()
        fp[i] += 1.0
        fm[i] -= 1.0
        fd = (loss(E0, fp) - loss(E0, fm)) / 2.0
        assert abs(fd - gf[i]) <= 1e-9 * np.abs(gf).max(), (i, fd, gf[i])
    h = 1e-6
    for e in p.extra["fd_elems"]:
        Ep, Em = E0.copy(), E0.copy()
        Ep[e] *= 1 + h
        Em[e] *= 1 - h
        fd = (loss(Ep, f0) - loss(Em, f0)) / (2 * h * E0[e])
        assert abs(fd - gE[e]) <= 1e-3 * np.abs(gE).max(), (e, fd, gE[e])
