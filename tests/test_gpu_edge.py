"""Edge cases and failure handling of the GPU path: a single-level hierarchy,
zero and non-finite loads, the iteration cap, a non-SPD matrix, a singular
matrix (free body), damping beyond 2/lambda_1 (PCG breakdown), repeatability,
and an extreme kappa_p that forces one interpolation entry per row (patterns
still bit-exact against the oracle)."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


def test_single_level(cuda):
    import torch
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(4)                       # 375 DOF: dense coarsest solve only
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0)
    assert S.nlev == 1
    u = S.solve(torch.tensor(p.f, device="cuda")).cpu().numpy()
    assert S.last_stats["iterations"] == 1 and S.last_stats["status"] == 0
    K = p.to_scipy().toarray()
    assert np.linalg.norm(K @ u - p.f) <= 1e-12 * np.linalg.norm(p.f)
    S.close()


@pytest.fixture(scope="module")
def cube(cuda):
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(7)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0)
    yield p, S
    S.close()


def test_zero_load(cube):
    import torch
    p, S = cube
    u = S.solve(torch.zeros(p.n_dof, dtype=torch.float64, device="cuda"))
    assert S.last_stats["status"] == 0 and S.last_stats["iterations"] == 0
    assert not u.any().item()


def test_nan_load(cube):
    import torch
    from paper_1902_01715_amd import aspamg
    p, S = cube
    f = torch.tensor(p.f, device="cuda")
    f[7] = float("nan")
    S.solve(f, check=False)
    assert S.last_stats["status"] == aspamg.ENAN


def test_iteration_cap(cuda):
    import torch
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(7)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(max_it=3))
    S.solve(torch.tensor(p.f, device="cuda"), check=False)
    st = S.last_stats
    assert st["status"] == aspamg.NOT_CONVERGED and st["iterations"] == 3
    S.close()


def test_non_spd_matrix_is_rejected(cuda):
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(7)
    vals = p.vals.copy()
    i = 200
    k = np.nonzero(p.col[p.row_ptr[i]:p.row_ptr[i + 1]] == i)[0][0] + p.row_ptr[i]
    vals[k] = -vals[k]
    with pytest.raises(aspamg.AspamgError) as e:
        aspamg.Solver(p.row_ptr, p.col, vals, p.V0)
    assert e.value.code == aspamg.ENOT_SPD


@pytest.mark.parametrize("prec", [64, 32])
def test_repeatable(cube, prec):
    import torch
    p, S = cube
    S.set_precision(prec)
    f = torch.tensor(p.f, device="cuda")
    u1 = S.solve(f).cpu().numpy()
    u2 = S.solve(f).cpu().numpy()
    assert np.array_equal(u1, u2)


def test_kappa_one_patterns_bit_exact(cuda, oracle_lib):
    import torch
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(10)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(kappa_p=1.0))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0, oracle_lib.default_params(kappa_p=1.0))
    assert S.nlev == H.nlev
    for l in range(H.nlev - 1):
        cf, cnt, cols = S.level_split(l)
        assert np.array_equal(cf, H.cf(l))
        cnt_o, cols_o = H.P_scalar(l)
        assert np.array_equal(cnt, cnt_o) and np.array_equal(cols, cols_o)
        assert cnt.mean() < 1.5               # kappa_p = 1 admits (almost always) one column per row
    u = S.solve(torch.tensor(p.f, device="cuda")).cpu().numpy()
    assert S.last_stats["status"] == 0
    u_o, _ = H.pcg(p.f, 1e-10, 1000)
    assert np.linalg.norm(u - u_o) / np.linalg.norm(u_o) <= 1e-8
    S.close()


def test_damping_beyond_two_over_lambda_breaks_pcg(cuda):
    """omega lambda_1(G A G^T) > 2 (a safety factor below 1 on the cantilever,
    whose fine level has lambda_1 = 2.44): the V-cycle is indefinite and the
    solve must stop with EBREAKDOWN, as the oracle does; the default margin
    converges."""
    import torch
    from paper_1902_01715_amd import aspamg
    print("[case omega beyond 2/lambda_1, cantilever 40x4x4]", flush=True)
    p = PR.c2_cantilever(40, 4, 4)
    f = torch.tensor(p.f, device="cuda")
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(omega_safety=0.6))
    li = S.level_info(0)
    assert li["omega_s"] * li["lambda1"] > 2.0
    for prec in (64, 32):
        S.set_precision(prec)
        with pytest.raises(aspamg.AspamgError) as ei:
            S.solve(f)
        assert ei.value.code == aspamg.EBREAKDOWN
    S.close()
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0)
    li = S.level_info(0)
    assert li["omega_s"] * li["lambda1"] < 2.0
    S.solve(f)
    assert S.last_stats["status"] == aspamg.OK
    S.close()


def test_singular_matrix_is_rejected(cuda):
    """A free body (no Dirichlet rows): K is singular and so is the coarsest
    Galerkin operator; setup must fail with ENOT_SPD (coarsest Cholesky)."""
    from paper_1902_01715_amd import aspamg
    print("[case singular K, free body 5^3]", flush=True)
    q = PR.unconstrained_box(5, 5, 5, seed=1)
    with pytest.raises(aspamg.AspamgError) as ei:
        aspamg.Solver(q.row_ptr, q.col, q.vals, q.V0)
    assert ei.value.code == aspamg.ENOT_SPD
    assert "coarsest" in str(ei.value)
