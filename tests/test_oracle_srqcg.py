"""Pins of the oracle's SRQCG test-space iteration (Section 3.3, Algorithm
"Test Space generation by SRQCG") against closed forms and textbook routines:
the spectrum of the 1D Laplacian, the Rayleigh-Ritz minimum over a
two-dimensional subspace, and a dense Cholesky solve of the whole method."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_1902_01715_amd import problems as PR


def _laplacian_1d(n):
    rp = np.zeros(n + 1, dtype=np.int64)
    ci, v = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                v.append(2.0 if i == j else -1.0)
        rp[i + 1] = len(ci)
    return rp, np.array(ci, dtype=np.int32), np.array(v).reshape(-1, 1, 1)


def _diag_factor(d):
    n = d.shape[0]
    return O.BSR(np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.reshape(-1, 1, 1).copy(), n, n, 1)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_srqcg_converges_to_laplacian_modes(seed, oracle_lib):
    """S = G A G^T with A = tridiag(-1, 2, -1) and G = I / sqrt(2) has the
    eigenvalues 1 - cos(k pi / (n + 1)) and the sine modes; with a Ritz
    projection every iteration the columns converge to the lowest four."""
    n, nt = 48, 4
    rp, ci, v = _laplacian_1d(n)
    G = _diag_factor(np.full(n, 1 / np.sqrt(2)))
    V0 = np.random.default_rng(seed).standard_normal((n, nt))
    V, rq = O.srqcg(rp, ci, v, G, V0, 120, 1, b=1)
    k = np.arange(1, nt + 1)
    exact = 1 - np.cos(k * np.pi / (n + 1))
    assert np.max(np.abs(rq - exact) / exact) < 1e-12
    modes = np.sin(np.outer(np.arange(1, n + 1), k) * np.pi / (n + 1))
    Qv, Qm = np.linalg.qr(V)[0], np.linalg.qr(modes)[0]
    assert np.linalg.svd(Qv.T @ Qm, compute_uv=False).min() > 1 - 1e-10
    # V = G^T Z: the columns of V are those of Z scaled by 1/sqrt(2); each
    # has the Rayleigh quotient of its eigenvalue
    for c in range(nt):
        z = V[:, c] * np.sqrt(2)
        S = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / 2
        assert abs(z @ S @ z / (z @ z) - exact[c]) <= 1e-12 * exact[c]


@pytest.mark.parametrize("seed", [4, 5])
def test_srqcg_step_is_the_line_minimum(seed, oracle_lib):
    """One update of one column (no projection) moves z to the minimiser of the
    Rayleigh quotient on the line z + t p, which is the Rayleigh-Ritz minimum
    over span{z, p}: the smallest eigenvalue of the 2 x 2 pencil."""
    n = 30
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    A = B @ B.T / n + np.diag(np.linspace(0.05, 2.0, n))
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    G = _diag_factor(1 / np.sqrt(np.diag(A)))
    Gd = np.diag(1 / np.sqrt(np.diag(A)))
    S = Gd @ A @ Gd.T
    v0 = rng.standard_normal((n, 1))
    V, rq = O.srqcg(rp, ci, A.reshape(-1, 1, 1), G, v0, 1, 10 ** 6, b=1)
    x0 = np.linalg.solve(Gd.T, v0[:, 0])          # V0 enters in the variable of S
    z0 = x0 - S @ x0
    z0 /= np.linalg.norm(z0)
    p0 = 2 * (S @ z0 - (z0 @ S @ z0) * z0)
    W = np.stack([z0, p0], axis=1)
    lam = sl.eigh(W.T @ S @ W, W.T @ W, eigvals_only=True)[0]
    assert abs(rq[0] - lam) <= 1e-12 * lam
    # and the returned column is G^T of a vector in span{z0, p0}
    z = np.linalg.solve(Gd.T, V[:, 0])
    resid = z - W @ np.linalg.lstsq(W, z, rcond=None)[0]
    assert np.linalg.norm(resid) <= 1e-12 * np.linalg.norm(z)


def test_srqcg_zero_iterations_is_the_smoothed_start(oracle_lib):
    """With k_max = 0 the result is G^T times the orthonormalised (I - S) X0,
    X0 = G^{-T} V0 the start vectors in the variable of S (dense solve)."""
    p = PR.c1_cube(7)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    assert H.nlev == 2
    G = H.G(0)
    V0 = PR.initial_test_space(p, 8, 7).reshape(p.n_dof, 8)
    V, _ = O.srqcg(p.row_ptr, p.col, p.vals, G, V0, 0, 1)
    Gd, A = G.to_dense(), p.to_scipy().toarray()
    X0 = np.linalg.solve(Gd.T, V0)
    Z0 = X0 - Gd @ A @ Gd.T @ X0
    Q = np.linalg.qr(Z0)[0]
    # the oracle orthonormalises by Cholesky-QR: the same columns up to signs
    # fixed by a positive triangular factor, i.e. Q with R's diagonal positive
    R = np.linalg.qr(Z0)[1]
    Q = Q * np.sign(np.diag(R))
    assert np.allclose(V, Gd.T @ Q, rtol=0, atol=1e-11 * np.abs(V).max())


@pytest.mark.parametrize("mk", [lambda: PR.c1_cube(8),
                                lambda: PR.box_problem("r", 7, 7, 7, 1, 1, 1,
                                                       E=10 ** np.random.default_rng(9).uniform(-3, 3, 343),
                                                       nu=0.3, clamp="z0", load=("body", (0, 0, -1)))])
def test_srqcg_hierarchy_solves(mk, oracle_lib):
    """The paper's test-space defaults (n_tv = 10, n_rq = 10, a Ritz projection
    every iteration) give a hierarchy whose PCG reaches the dense solution;
    every level's test space is orthonormal."""
    p = mk()
    V0 = PR.initial_test_space(p, 10, 11)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, V0, O.default_params(n_rq=10))
    assert H.nlev >= 2
    u, st = H.pcg(p.f, 1e-10, 500)
    assert st["status"] == 0
    K = p.to_scipy().toarray()
    us = sl.cho_solve(sl.cho_factor(K), p.f)
    assert np.linalg.norm(u - us) / np.linalg.norm(us) <= 1e-8
    for l in range(H.nlev - 1):
        V = H.V(l)
        Vm = V.reshape(-1, V.shape[-1])
        keep = np.abs(Vm).max(axis=0) > 0
        assert np.allclose(Vm[:, keep].T @ Vm[:, keep], np.eye(keep.sum()), atol=1e-10)


def test_srqcg_converges_on_elasticity(oracle_lib):
    """On the 7^3 elasticity cube with its own aFSAI factor G (b = 3), the
    columns converge to the four smallest eigenpairs of S = G A G^T computed
    by a dense symmetric eigensolver: Ritz values to 1e-11 and V = G^T Z
    spanning G^T of the eigenvectors."""
    p = PR.c1_cube(7)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    G = H.G(0)
    Gd, A = G.to_dense(), p.to_scipy().toarray()
    S = Gd @ A @ Gd.T
    w, X = np.linalg.eigh((S + S.T) / 2)
    V0 = np.random.default_rng(3).standard_normal((p.n_dof, 4))
    V, rq = O.srqcg(p.row_ptr, p.col, p.vals, G, V0, 100, 1)
    assert np.max(np.abs(rq - w[:4]) / w[:4]) < 1e-11
    Qv = np.linalg.qr(V)[0]
    Qe = np.linalg.qr(Gd.T @ X[:, :4])[0]
    assert np.linalg.svd(Qv.T @ Qe, compute_uv=False).min() > 1 - 1e-8


@pytest.mark.parametrize("kmax", [0, 6])
def test_srqcg_keeps_the_rigid_body_modes_of_a_free_body(kmax, oracle_lib):
    """On an unconstrained (singular) elasticity K the rigid-body modes span its
    kernel.  Entering in the variable of S as G^{-T} V0, they lie in the kernel
    of S = G A G^T (S G^{-T} V0 = G A V0 = 0), so neither the smoothing step nor
    the Rayleigh-quotient iteration moves them: V = G^T Z spans the modes
    again.  G is the FSAI factor on the lower block pattern of K."""
    p = PR.unconstrained_box(4, 4, 3, jitter=0.2, seed=1)
    n = p.n_nodes
    brp, bci = [0], []
    for i in range(n):
        row = p.col[p.row_ptr[i]:p.row_ptr[i + 1]]
        bci.extend(int(j) for j in row if j < i)
        brp.append(len(bci))
    G, _ = O.fsai_fixed(p.row_ptr, p.col, p.vals, np.array(brp), np.array(bci, dtype=np.int32))
    R = p.V0.reshape(p.n_dof, 6)
    V, rq = O.srqcg(p.row_ptr, p.col, p.vals, G, R, kmax, 1)
    Q = np.linalg.qr(R)[0]
    resid = V - Q @ (Q.T @ V)
    assert np.linalg.norm(resid) <= 1e-9 * np.linalg.norm(V)
    assert np.linalg.matrix_rank(V, tol=1e-8 * np.abs(V).max()) == 6
