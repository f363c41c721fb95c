"""GPU set-up with the SRQCG test space (Section 3.3, Algorithm "Test Space
generation by SRQCG"; n_tv = 10, n_rq = 10, a Ritz projection every
iteration) against the oracle on the same seeded inputs.

Both sides take the iteration's inner products in one fixed order (blocks of
256 entries, then the block sums) and its products with G, A and G^T row by
row in stored order, so each level's test space is bit for bit the oracle's,
and so are the C/F split, the interpolation pattern and its weights; the
solution agrees to the solve tolerance."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu

CASES = {
    "cube8": lambda: PR.c1_cube(8),
    "cube8_randE": lambda: PR.box_problem("r", 8, 8, 8, 1, 1, 1, E=10 ** np.random.default_rng(7).uniform(-3, 3, 512),
                                          nu=0.3, clamp="z0", load=("body", (0, 0, -1))),
    "cube12": lambda: PR.c1_cube(12),
    "cube16": lambda: PR.c1_cube(16),
}

@pytest.fixture(scope="module", params=list(CASES))
def srq_pair(request, cuda, oracle_lib):
    from paper_1902_01715_amd import aspamg
    name = request.param
    print(f"[srqcg case {name}]", flush=True)
    p = CASES[name]()
    V0 = PR.initial_test_space(p, 10, 11)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, V0, aspamg.default_params(n_rq=10))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, V0, oracle_lib.default_params(n_rq=10))
    yield name, p, S, H
    S.close()


def test_srqcg_test_space_and_split(srq_pair):
    name, p, S, H = srq_pair
    assert S.nlev == H.nlev, (S.nlev, H.nlev)
    for l in range(H.nlev - 1):
        Vg = S.level_test_space(l).reshape(-1, 10)
        Vo = H.V(l).reshape(-1, 10)
        cf_g, cnt_g, cols_g = S.level_split(l)
        cf_o = H.cf(l)
        print(f"{name} level {l}: |V_g - V_o|max {np.abs(Vg - Vo).max():.2e}, "
              f"C/F differ at {int((cf_g != cf_o).sum())} of {cf_o.size} nodes", flush=True)
        assert np.array_equal(Vg, Vo), l
        assert np.array_equal(cf_g, cf_o), l
        cnt_o, cols_o = H.P_scalar(l)
        assert np.array_equal(cnt_g, cnt_o) and np.array_equal(cols_g, cols_o), l
        P_g, P_o = S.level_matrix(l, 3), H.P(l)
        assert np.array_equal(P_g[1], P_o.ci) and np.array_equal(P_g[2], P_o.v), l
        A_g, A_o = S.level_matrix(l + 1, 0), H.A(l + 1)
        assert np.array_equal(A_g[2], A_o.v), l


@pytest.mark.parametrize("prec", [64, 32])
def test_srqcg_solve_matches_oracle(srq_pair, prec):
    import torch
    name, p, S, H = srq_pair
    u_o, st_o = H.pcg(p.f, 1e-10, 1000)
    assert st_o["status"] == 0
    S.set_precision(prec)
    u = S.solve(torch.tensor(p.f, device="cuda")).cpu().numpy()
    st = S.last_stats
    err = np.linalg.norm(u - u_o) / np.linalg.norm(u_o)
    print(f"{name} prec={prec} it={st['iterations']} (oracle {st_o['iterations']}) err={err:.2e} "
          f"true res {st['relres_true']:.2e}")
    assert st["status"] == 0, st
    assert st["relres_true"] <= 2e-10
    assert err <= 1e-8, err


@pytest.mark.parametrize("n_tv,n_rq", [(1, 3), (6, 5)])
def test_srqcg_few_test_vectors(n_tv, n_rq, cuda, oracle_lib):
    """One test vector (a single column: the smallest batch of inner products
    is the column update's five) and the six rigid-body modes without padding."""
    import torch
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(8)
    V0 = np.ascontiguousarray(p.V0[:, :, :n_tv])
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, V0, aspamg.default_params(n_rq=n_rq))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, V0, oracle_lib.default_params(n_rq=n_rq))
    try:
        assert S.nlev == H.nlev
        Vg, Vo = S.level_test_space(0).reshape(-1, n_tv), H.V(0).reshape(-1, n_tv)
        assert np.array_equal(Vg, Vo)
        assert np.array_equal(S.level_split(0)[0], H.cf(0))
        u_o, st_o = H.pcg(p.f, 1e-10, 1000)
        u = S.solve(torch.tensor(p.f, device="cuda")).cpu().numpy()
        assert S.last_stats["status"] == 0
        assert np.linalg.norm(u - u_o) / np.linalg.norm(u_o) <= 1e-8
    finally:
        S.close()
