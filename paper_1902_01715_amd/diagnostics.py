"""Smoother-quality diagnostics of Section 3.2 ("Influence of omega on the AMG
cycle") for small hierarchies (a few thousand unknowns per level).

The setup products come from the library: A_l, G_l and P_l through
aspamg_level_matrix, the Lanczos estimate lambda_hat_1 and the applied damping
omega_s through aspamg_level_info, and the whole V-cycle through aspamg_vcycle
applied on the device to the columns of the identity.  Spectra are dense
symmetric eigensolves of those exports on the host (this is an analysis tool
next to the solver, not part of the solve path).

  level_report(S, l)   lambda_1(G A G^T) exact against the Lanczos estimate,
                       omega_q = 2 / lambda_hat_1, the smoother's spectral
                       radius rho(I - omega_s G^T G A) and the two-grid error
                       propagation E_TG = S (I - P A_c^{-1} P^T A) S of the
                       level (Section 2, eq. (twoGridErrorOp)) with its
                       spectral radius in the energy norm
  vcycle_report(S)     E_V = I - B A of the library's V-cycle B on the finest
                       level: spectral radius and the extreme eigenvalues of B A
  s_alpha_report(S)    the low-rank experiment of Section 3.2: the smoother
                       M_alpha = G^T G + alpha G^T U U^T G^{-T} A^{-1} with U the
                       top eigenvectors of G A G^T keeps the hierarchy but
                       moves the top of the spectrum; its largest admissible
                       damping is 2 omega / (2 + alpha omega); two-grid
                       spectral radius and stationary AMG iterations with the
                       original and the updated smoother

    python -m paper_1902_01715_amd.diagnostics      # cube 7^3 and a layered block
"""
from __future__ import annotations

import numpy as np


def bsr_dense(M, ncols=None):
    """Dense matrix of an exported block matrix (row_ptr, col, [nnzb,3,3])."""
    rp, ci, v = M
    n = rp.size - 1
    nc = ncols if ncols is not None else n
    D = np.zeros((3 * n, 3 * nc))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = ci[k]
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = v[k]
    return D


def _energy_sym(E, L):
    """Eigenvalues of the A-self-adjoint E through its symmetric form L^T E L^{-T} (A = L L^T)."""
    T = L.T @ E @ np.linalg.inv(L.T)
    return np.linalg.eigvalsh(0.5 * (T + T.T))


def two_grid(A, G, P, omega, Ac=None):
    """E_TG = (I - omega G^T G A)(I - P Ac^{-1} P^T A)(I - omega G^T G A)."""
    n = A.shape[0]
    Ac = P.T @ A @ P if Ac is None else Ac
    S = np.eye(n) - omega * (G.T @ G) @ A
    C = np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)
    return S @ C @ S


def stationary_iterations(A, E, tol=1e-8, max_it=5000):
    """Iterations of x <- x + B (b - A x) from x = 0 with b = 1 (the paper's
    right-hand side) until ||b - A x|| <= tol ||b||; B = (I - E) A^{-1}."""
    n = A.shape[0]
    b = np.ones(n)
    B = (np.eye(n) - E) @ np.linalg.inv(A)
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    for k in range(1, max_it + 1):
        x = x + B @ (b - A @ x)
        if np.linalg.norm(b - A @ x) <= tol * nb:
            return k
    return max_it + 1


def _free(S, level):
    """Unknowns of the level that are not decoupled (constrained) rows."""
    cf = S.level_split(level)[0] if S.level_info(level)["n_coarse"] > 0 else None
    n = S.level_info(level)["n"]
    if cf is None:
        return np.ones(3 * n, dtype=bool)
    return np.repeat(cf >= 0, 3)


def level_report(S, level):
    li = S.level_info(level)
    if not li["has_smoother"]:
        raise ValueError("the coarsest level has no smoother")
    A = bsr_dense(S.level_matrix(level, 0))
    G = bsr_dense(S.level_matrix(level, 1))
    P = bsr_dense(S.level_matrix(level, 3), li["n_coarse"])
    Ac = bsr_dense(S.level_matrix(level + 1, 0))
    lam = np.linalg.eigvalsh(0.5 * (G @ A @ G.T + (G @ A @ G.T).T))
    keep = _free(S, level)
    Af = A[np.ix_(keep, keep)]
    E = two_grid(A, G, P, li["omega_s"], Ac)[np.ix_(keep, keep)]
    L = np.linalg.cholesky(Af)
    mu = _energy_sym(E, L)
    return {"level": level, "n_dof": A.shape[0], "lambda1": lam[-1], "lambda1_lanczos": li["lambda1"],
            "lanczos_rel_gap": (lam[-1] - li["lambda1"]) / lam[-1], "lambda_min": lam[0],
            "omega_q": li["omega_q"], "omega_s": li["omega_s"], "omega_s_lambda1": li["omega_s"] * lam[-1],
            "rho_smoother": float(np.max(np.abs(1.0 - li["omega_s"] * lam))),
            "rho_two_grid": float(np.max(np.abs(mu)))}


def vcycle_report(S, precision=64):
    """E_V = I - B A of the library's V-cycle on the finest level."""
    import torch
    A = bsr_dense(S.level_matrix(0, 0))
    n = A.shape[0]
    S.set_precision(precision)
    B = np.zeros((n, n))
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    for j in range(n):
        B[:, j] = S.vcycle(eye[:, j].contiguous()).cpu().numpy()
    keep = _free(S, 0)
    Af, Bf = A[np.ix_(keep, keep)], B[np.ix_(keep, keep)]
    L = np.linalg.cholesky(Af)
    BA = L.T @ Bf @ L                       # similar to B A, symmetric when B is
    sym_err = float(np.abs(BA - BA.T).max() / np.abs(BA).max())
    w = np.linalg.eigvalsh(0.5 * (BA + BA.T))
    return {"n_dof": n, "levels": S.nlev, "B_symmetry_error": sym_err, "lambda_min_BA": float(w[0]),
            "lambda_max_BA": float(w[-1]), "kappa_BA": float(w[-1] / w[0]),
            "rho_vcycle": float(np.max(np.abs(1.0 - w))), "B": B}


def s_alpha_report(S, alpha=5.0, k=10, level=0):
    """Section 3.2's low-rank update of the smoother on one level.  With U the
    k top eigenvectors of G A G^T (eigenvalues Lambda_U),
    M_alpha = G^T G + alpha G^T U U^T G^{-T} A^{-1} = G^T (I + alpha U Lambda_U^{-1} U^T) G
    is symmetric, and M_alpha A = G^T (G A G^T + alpha U U^T) G^{-T} has the
    eigenvectors of the original with the top k eigenvalues raised by alpha:
    the largest admissible damping falls from omega = 2 / lambda_1 to
    2 omega / (2 + alpha omega).  Both smoothers are applied with the library's
    rule min(1, 2 / (safety lambda_max)) in the two-grid cycle of the level."""
    li = S.level_info(level)
    A = bsr_dense(S.level_matrix(level, 0))
    G = bsr_dense(S.level_matrix(level, 1))
    P = bsr_dense(S.level_matrix(level, 3), li["n_coarse"])
    Ac = bsr_dense(S.level_matrix(level + 1, 0))
    keep = _free(S, level)
    GAG = G @ A @ G.T
    lam, U = np.linalg.eigh(0.5 * (GAG + GAG.T))
    omega = 2.0 / lam[-1]
    U, lamU = U[:, -k:], lam[-k:]
    M_alpha = G.T @ G + alpha * G.T @ U @ U.T @ np.linalg.inv(G).T @ np.linalg.inv(A)
    M_alpha = 0.5 * (M_alpha + M_alpha.T)
    lam_alpha = float(np.max(np.linalg.eigvals(M_alpha @ A).real))
    out = {"alpha": alpha, "k": k, "omega": omega, "omega_alpha_closed_form": 2.0 * omega / (2.0 + alpha * omega),
           "omega_alpha_dense": 2.0 / lam_alpha,
           "symmetric_form_error": float(np.abs(M_alpha - G.T @ (np.eye(A.shape[0]) + alpha * U @ np.diag(1 / lamU)
                                                                 @ U.T) @ G).max() / np.abs(M_alpha).max())}
    n = A.shape[0]
    C = np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)
    Af = A[np.ix_(keep, keep)]
    L = np.linalg.cholesky(Af)
    safety = S.params.omega_safety
    for name, M, lmax in (("original", G.T @ G, lam[-1]), ("updated", M_alpha, lam_alpha)):
        w = min(1.0, 2.0 / (safety * lmax))
        Sm = np.eye(n) - w * M @ A
        E = (Sm @ C @ Sm)[np.ix_(keep, keep)]
        mu = _energy_sym(E, L)
        out[name] = {"damping": w, "rho_two_grid": float(np.max(np.abs(mu))),
                     "stationary_iterations": stationary_iterations(Af, E)}
    return out


def _demo():
    import json
    from . import aspamg, problems as PR
    for name, p in (("cube 7^3", PR.c1_cube(7)),
                    ("layered 12x12x8", PR.c3_layered_distorted(12, 12, 8))):
        S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=0))
        rep = {"problem": name, "levels": [level_report(S, l) for l in range(S.nlev - 1)]}
        v = vcycle_report(S)
        v.pop("B")
        rep["vcycle"] = v
        rep["s_alpha"] = s_alpha_report(S)
        print(json.dumps(rep, indent=1, default=float))
        S.close()


if __name__ == "__main__":
    _demo()
