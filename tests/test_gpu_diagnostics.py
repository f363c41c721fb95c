"""Section 3.2 diagnostics (paper_1902_01715_amd.diagnostics) on the 7^3 cube,
whose hierarchy has two levels (the dense tail off, so the V-cycle is the
sparse one):

  - lambda_1(G A G^T) by a dense eigensolve against the library's Lanczos
    estimate (below it, within 1e-3), omega_s lambda_1 < 2, a convergent
    smoother and two-grid cycle;
  - the two-grid spectral radius equals the one computed here from the
    oracle's own matrices with eq. (twoGridErrorOp);
  - with two levels the library's V-cycle B, applied on the GPU to the columns
    of the identity, is the dense two-grid operator (I - E_TG) A^{-1} of the
    oracle's matrices;
  - the low-rank update of Section 3.2: the largest admissible damping of the
    updated smoother is 2 omega / (2 + alpha omega), and the updated two-grid
    cycle converges more slowly (larger spectral radius, more stationary
    iterations), the paper's observation."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube(cuda, oracle_lib):
    from paper_1902_01715_amd import aspamg
    print("[case diagnostics cube 7^3]", flush=True)
    p = PR.c1_cube(7)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=0))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    assert S.nlev == 2 and H.nlev == 2
    yield p, S, H
    S.close()


def oracle_two_grid(H):
    A, G, P, Ac = H.A(0).to_dense(), H.G(0).to_dense(), H.P(0).to_dense(), H.A(1).to_dense()
    n = A.shape[0]
    w = H.info(0)["omega_s"]
    Sm = np.eye(n) - w * G.T @ G @ A
    E = Sm @ (np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)) @ Sm
    return A, E


def test_level_report(cube):
    from paper_1902_01715_amd import diagnostics as D
    p, S, H = cube
    r = D.level_report(S, 0)
    assert 0.0 <= r["lanczos_rel_gap"] <= 1e-3, r
    assert r["omega_s_lambda1"] < 2.0 and r["rho_smoother"] < 1.0 and r["rho_two_grid"] < 1.0
    A, E = oracle_two_grid(H)
    free = ~np.repeat(p.dirichlet, 3)
    Ef = E[np.ix_(free, free)]
    L = np.linalg.cholesky(A[np.ix_(free, free)])
    mu = np.linalg.eigvals(L.T @ Ef @ np.linalg.inv(L.T))
    assert abs(r["rho_two_grid"] - np.abs(mu).max()) <= 1e-10
    print(r, flush=True)


def test_vcycle_is_the_two_grid_operator(cube):
    from paper_1902_01715_amd import diagnostics as D
    p, S, H = cube
    v = D.vcycle_report(S)
    A, E = oracle_two_grid(H)
    free = ~np.repeat(p.dirichlet, 3)
    B_ref = (np.eye(A.shape[0]) - E) @ np.linalg.inv(A)
    Bf, Rf = v["B"][np.ix_(free, free)], B_ref[np.ix_(free, free)]
    assert np.abs(Bf - Rf).max() <= 1e-10 * np.abs(Rf).max()
    assert v["B_symmetry_error"] <= 1e-12
    assert 0.0 < v["lambda_min_BA"] and v["lambda_max_BA"] <= 1.0 + 1e-10
    print({k: v[k] for k in v if k != "B"}, flush=True)


def test_s_alpha_experiment(cube):
    from paper_1902_01715_amd import diagnostics as D
    p, S, H = cube
    r = D.s_alpha_report(S, alpha=5.0, k=10)
    assert abs(r["omega_alpha_dense"] - r["omega_alpha_closed_form"]) <= 1e-9 * r["omega_alpha_closed_form"]
    assert r["symmetric_form_error"] <= 1e-10
    assert r["updated"]["damping"] < r["original"]["damping"]
    assert r["updated"]["rho_two_grid"] > r["original"]["rho_two_grid"]
    assert r["updated"]["stationary_iterations"] > r["original"]["stationary_iterations"]
    print(r, flush=True)
