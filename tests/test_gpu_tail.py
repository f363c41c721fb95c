"""The small levels of the V-cycle.  The dense tail: the V-cycle from the
highest level whose unknowns, and those of every level below it, number at
most `dense_tail_dof` is formed at setup as one dense FP64 operator.  It is the same linear operator as the sparse cycle
of those levels, so the V-cycle, the solve and the iteration counts must agree
with the all-sparse cycle and the oracle up to rounding; the V-cycle stays
symmetric (symmetric smoother, Galerkin coarse operators, nu1 = nu2).  Small
smoothed levels above the tail store M = G^T G and apply it in one product."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def layered(cuda, oracle_lib):
    from paper_1902_01715_amd import aspamg
    p = PR.c3_layered_distorted(32, 32, 16)   # 55,539 DOF, 4 levels
    print("[case layered 32x32x16 tail/sparse]", flush=True)
    St = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0)
    Ss = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=0))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    yield p, St, Ss, H
    St.close()
    Ss.close()


def _expected_tail(S, dof):
    sizes = [3 * S.level_info(l)["n"] for l in range(S.nlev)]
    t = S.nlev - 1
    while t > 0 and sizes[t - 1] <= dof:
        t -= 1
    return -1 if t == S.nlev - 1 else t


def test_tail_level(layered):
    import torch
    p, St, Ss, _ = layered
    f = torch.tensor(p.f, device="cuda")
    St.solve(f, check=False)
    Ss.solve(f, check=False)
    t = St.last_stats["tail_level"]
    assert t == _expected_tail(St, 4096) and 0 < t < St.nlev - 1, t
    assert Ss.last_stats["tail_level"] == -1


@pytest.mark.parametrize("prec", [64, 32])
def test_tail_cycle_matches_sparse_cycle(layered, prec):
    import torch
    p, St, Ss, H = layered
    rng = np.random.default_rng(21)
    y = rng.standard_normal(3 * St.level_info(0)["n"])
    St.set_precision(prec)
    Ss.set_precision(prec)
    zt = St.vcycle(torch.tensor(y, device="cuda")).cpu().numpy()
    zs = Ss.vcycle(torch.tensor(y, device="cuda")).cpu().numpy()
    zo = H.vcycle(y)
    d_ts = np.linalg.norm(zt - zs) / np.linalg.norm(zs)
    d_to = np.linalg.norm(zt - zo) / np.linalg.norm(zo)
    print(f"prec {prec}: tail vs sparse {d_ts:.2e}, tail vs oracle {d_to:.2e}", flush=True)
    # FP64: both are the oracle's operator to rounding; FP32: the sparse cycle
    # rounds levels t.. in FP32, the tail applies them in FP64
    bar = 1e-11 if prec == 64 else 1e-4
    assert d_ts <= bar and d_to <= bar
    St.set_precision(64)
    Ss.set_precision(64)


def test_tail_cycle_is_symmetric(layered):
    import torch
    _, St, _, _ = layered
    n = 3 * St.level_info(0)["n"]
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    St.set_precision(64)
    Bx = St.vcycle(torch.tensor(x, device="cuda")).cpu().numpy()
    By = St.vcycle(torch.tensor(y, device="cuda")).cpu().numpy()
    a, b = y @ Bx, x @ By
    assert abs(a - b) <= 1e-11 * np.sqrt(abs(x @ Bx) * abs(y @ By))


def test_tail_solve_matches_oracle(layered):
    import torch
    p, St, Ss, H = layered
    uo, sto = H.pcg(p.f, 1e-10, 1000)
    for S in (St, Ss):
        for prec in (64, 32):
            S.set_precision(prec)
            u = S.solve(torch.tensor(p.f, device="cuda"), check=False).cpu().numpy()
            st = S.last_stats
            err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
            print(f"tail {st['tail_level']} prec {prec}: it {st['iterations']} (oracle {sto['iterations']}) "
                  f"err {err:.2e}", flush=True)
            assert st["status"] == 0 and err <= 1e-8
            if prec == 64:
                assert abs(st["iterations"] - sto["iterations"]) <= 1
        S.set_precision(64)


def test_tail_parameter_bounds(cuda):
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(5)
    with pytest.raises(aspamg.AspamgError):
        aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=8193))
    with pytest.raises(aspamg.AspamgError):
        aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=-1))


def test_merged_smoother_is_gtg(layered, product_bound):
    import scipy.sparse as sp
    import torch
    _, St, Ss, _ = layered
    merged = [l for l in range(St.nlev) if St.level_info(l)["nnzb_M"] > 0]
    # the 4,131-node level 1 of the layered block merges; the 18,513-node fine level does not
    assert merged == [1] and Ss.level_info(1)["nnzb_M"] > 0 and St.level_info(0)["nnzb_M"] == 0
    li = St.level_info(1)
    rp, ci, v = St.level_matrix(1, 1)
    G = sp.bsr_matrix((v, ci, rp), shape=(3 * li["n"], 3 * li["n"])).tocsr()
    # blocks of G^T G: the node pattern of G (ones) squared, no cancellation possible
    Gn = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(li["n"], li["n"]))
    assert li["nnzb_M"] == (Gn.T @ Gn).nnz
    rng = np.random.default_rng(8)
    x = rng.standard_normal(3 * li["n"])
    ref = G.T @ (G @ x)
    for prec in (64, 32):
        y = St.apply(1, 5, torch.tensor(x, device="cuda"), precision=prec).cpu().numpy()
        # M's entries are sums over G's blocks: bound the two-stage product
        bound = product_bound(abs(G).T @ abs(G), np.abs(x), prec) * 4
        assert np.all(np.abs(y - ref) <= bound + 1e-300), prec


def test_tail_over_two_smoothed_levels(cuda, oracle_lib):
    """dense_tail_dof = 8192 on the 12^3 cube (6,591 / 2,019 / 441 DOF) folds the
    whole cycle, two smoothed levels and the coarsest, into one dense operator."""
    import torch
    from paper_1902_01715_amd import aspamg
    p = PR.c1_cube(12)
    print("[case cube 12^3 tail 8192]", flush=True)
    S8 = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=8192))
    S0 = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(dense_tail_dof=0))
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    assert S8.nlev == H.nlev == 3
    f = torch.tensor(p.f, device="cuda")
    rng = np.random.default_rng(12)
    y = rng.standard_normal(p.f.shape[0])
    z8 = S8.vcycle(torch.tensor(y, device="cuda")).cpu().numpy()
    z0 = S0.vcycle(torch.tensor(y, device="cuda")).cpu().numpy()
    zo = H.vcycle(y)
    assert np.linalg.norm(z8 - z0) <= 1e-11 * np.linalg.norm(z0)
    assert np.linalg.norm(z8 - zo) <= 1e-11 * np.linalg.norm(zo)
    uo, sto = H.pcg(p.f, 1e-10, 1000)
    u = S8.solve(f, check=False).cpu().numpy()
    st = S8.last_stats
    assert st["tail_level"] == 0 and st["status"] == 0
    assert abs(st["iterations"] - sto["iterations"]) <= 1
    assert np.linalg.norm(u - uo) <= 1e-8 * np.linalg.norm(uo)
    S8.close()
    S0.close()
