"""Pins of the synthetic FE input generator (Q1 elasticity, Section 1 eq. (1)).

The stiffness matrix is checked against what mechanics fixes: symmetry, the six
rigid-body modes as the null space of the unconstrained operator, the patch
test, consistent-load totals and the Euler-Bernoulli/Timoshenko cantilever."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse.linalg as spl

from paper_1902_01715_amd import problems as PR


def test_c1_counts_and_exact_symmetry():
    p = PR.c1_cube(10)
    assert p.n_nodes == 1331 and p.n_dof == 3993 and p.nnzb == 27029
    assert p.dirichlet.sum() == 121
    K = p.to_scipy()
    assert (K - K.T).count_nonzero() == 0          # bitwise symmetric
    # clamped rows are identity, with no coupling blocks
    for i in np.nonzero(p.dirichlet)[0][:5]:
        assert p.row_ptr[i + 1] - p.row_ptr[i] == 1
        assert np.array_equal(p.vals[p.row_ptr[i]], np.eye(3))


def test_c5_counts():
    rp, col, _ = PR.structured_pattern(48, 48, 48, (np.arange(49 ** 3) // 49 ** 2) == 0)
    assert rp.size - 1 == 117649 and rp[-1] == 2987951


def test_element_has_six_rigid_modes():
    rng = np.random.default_rng(0)
    X = PR._SIGNS * 0.5 + 0.08 * rng.standard_normal((8, 3))
    Ke = PR.element_stiffness(X[None], *PR.lame(2.0, 0.3))[0]
    w = np.linalg.eigvalsh((Ke + Ke.T) / 2)
    assert np.all(np.abs(w[:6]) < 1e-12 * w[-1])
    assert np.all(w[6:] > 1e-6 * w[-1])


def test_unconstrained_K_annihilates_rigid_body_modes():
    p = PR.unconstrained_box(3, 2, 4, 1.0, 0.7, 1.3, jitter=0.3, seed=5)
    K = p.to_scipy()
    V = p.V0.reshape(-1, 6)
    R = K @ V
    assert np.abs(R).max() <= 1e-12 * abs(K).max() * np.abs(V).max()


def test_patch_test_on_jittered_mesh():
    """A linear displacement field prescribed on the boundary is reproduced inside."""
    p = PR.unconstrained_box(4, 4, 4, jitter=0.3, seed=1)
    K = p.to_scipy().toarray()
    a = np.array([0.1, -0.2, 0.3])
    B = np.array([[0.01, 0.02, -0.03], [0.04, -0.01, 0.02], [-0.02, 0.03, 0.05]])
    u_lin = (a[None, :] + p.coords @ B.T).reshape(-1)
    bnd = np.repeat(PR.boundary_node_mask(4, 4, 4), 3)
    inn = ~bnd
    u = u_lin.copy()
    u[inn] = np.linalg.solve(K[np.ix_(inn, inn)], -K[np.ix_(inn, bnd)] @ u_lin[bnd])
    assert np.abs(u - u_lin).max() <= 1e-12 * np.abs(u_lin).max()


def test_consistent_load_totals():
    p = PR.box_problem("b", 3, 4, 5, 1.5, 2.0, 0.5, E=1.0, nu=0.3, clamp=None, load=("body", (1.0, -2.0, 3.0)))
    assert np.allclose(p.f.reshape(-1, 3).sum(0), np.array([1.0, -2.0, 3.0]) * 1.5 * 2.0 * 0.5, rtol=1e-13)
    q = PR.box_problem("t", 4, 3, 2, 2.0, 0.6, 0.4, E=1.0, nu=0.3, clamp=None,
                       load=("traction", "x1", (0.0, 0.5, -1.0)))
    assert np.allclose(q.f.reshape(-1, 3).sum(0), np.array([0.0, 0.5, -1.0]) * 0.6 * 0.4, rtol=1e-13)


def test_cantilever_tip_deflection_beam_theory():
    """nu = 0 cantilever, L/H = 20: tip deflection within 5% of PL^3/(3EI) + PL/(kGA)."""
    H, L, E = 1.0, 20.0, 1.0
    nx, ny, nz = 160, 8, 8
    p = PR.box_problem("eb", nx, ny, nz, L, H, H, E=E, nu=0.0, clamp="x0",
                       load=("traction", "x1", (0.0, 0.0, -1.0)))
    K = p.to_scipy().tocsc()
    u = spl.spsolve(K, p.f).reshape(-1, 3)
    tip = np.isclose(p.coords[:, 0], L)
    w = -u[tip, 2].mean()
    P = H * H
    I = H ** 4 / 12.0
    G = E / 2.0
    w_ref = P * L ** 3 / (3 * E * I) + P * L / ((5.0 / 6.0) * G * H * H)
    assert abs(w - w_ref) / w_ref < 0.05, (w, w_ref)


# ----------------------------------------------------------------------------- P1 tetrahedra (block size 1)
def test_tet_mesh_fills_the_box_with_positive_volumes():
    coords, tets = PR.tet_mesh(3, 4, 2, jitter=0.25, seed=5)
    g, vol = PR._tet_gradients(coords[tets])
    assert tets.shape == (6 * 3 * 4 * 2, 4)
    assert (vol > 0).all() and abs(vol.sum() - 1.0) < 1e-13
    # every interior face is shared by exactly two tetrahedra, boundary faces by one
    faces = np.sort(tets[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(counts.tolist()) <= {1, 2}
    # barycentric gradients: sum to zero, and reproduce linear fields exactly
    assert np.abs(g.sum(axis=1)).max() < 1e-12
    lin = coords @ np.array([0.3, -1.2, 2.0])
    assert np.allclose(np.einsum("ea,eak->ek", lin[tets], g), [0.3, -1.2, 2.0], atol=1e-12)


def test_tet_diffusion_is_spd_with_constant_kernel_and_total_load():
    p = PR.tet_diffusion(4, 4, 3, contrast=1e2, layers=2, seed=1)
    A = p.to_scipy().toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
    assert np.allclose(p.vals.shape[1:], (1, 1))
    free = ~p.dirichlet
    # rows away from the clamped face annihilate the constant (the kernel of the Neumann operator)
    far = free & (p.coords[:, 2] > 0.4)
    assert np.abs((A @ np.ones(p.n))[far]).max() <= 1e-12 * np.abs(A).max()
    # f = integral of the unit source over the box, minus the clamped nodes' share
    assert 0.0 < p.f.sum() < 1.0 and np.all(p.f[p.dirichlet] == 0.0)


def test_tet_elasticity_rigid_modes_and_patch():
    p = PR.tet_elasticity(3, 3, 3, seed=2)
    K = p.to_scipy().toarray()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    assert np.linalg.eigvalsh(K).min() > 0
    # rows whose element neighbourhood avoids the clamped face annihilate the rigid-body modes
    nodes_far = p.coords[:, 2] > 0.5
    rows = np.repeat(nodes_far, 3)
    V = p.V0.reshape(p.n, 6)
    assert np.abs((K @ V)[rows]).max() <= 1e-11 * np.abs(K).max()
    # a linear displacement field has the same strain in every tetrahedron
    Gm = np.array([[0.1, 0.0, -0.2], [0.3, 0.2, 0.0], [0.0, -0.1, 0.4]])
    u_lin = p.coords @ Gm                              # u_i = sum_k x_k Gm[k, i]
    g, _ = PR._tet_gradients(p.coords[p.tets])
    grad = np.einsum("eai,eak->eik", u_lin[p.tets], g)  # du_i / dx_k per element
    assert np.allclose(grad, Gm.T[None], atol=1e-12)
