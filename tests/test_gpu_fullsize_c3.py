"""Full-size checks on the layered distorted block (128x128x64 Q1, 3,244,995 DOF)
in the launch configuration the benchmark times (FP32 and FP64 cycle):
FSAI rows of sampled block rows recomputed by the oracle row by row (pattern
and values bit for bit), and the solve's recursive and true residuals."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3(cuda):
    from paper_1902_01715_amd import aspamg
    print("[case c3 full size]", flush=True)
    p = PR.c3_layered_distorted()
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(max_it=60))
    yield p, S
    S.close()


def test_c3_sampled_fsai_rows_bit_exact(c3, oracle_lib):
    p, S = c3
    assert S.level_info(0)["fsai_rounds"] == 0
    rp, ci, v = S.level_matrix(0, 1)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(p.n_nodes, 400, replace=False)).astype(np.int32)
    pats, g, psi = oracle_lib.fsai_rows(oracle_lib.default_params(), oracle_lib.problem_rp(p), p.col, p.vals, rows)
    for r, I in enumerate(rows):
        nodes = ci[rp[I]:rp[I + 1]]
        assert np.array_equal(nodes[:-1], pats[r]) and nodes[-1] == I, I
        nb = len(pats[r])
        blocks = v[rp[I]:rp[I + 1]]
        for d in range(3):
            ref = g[r, d, :3 * nb + d + 1]
            got = np.concatenate([blocks[:nb, d, :].reshape(-1), blocks[nb, d, :d + 1]])
            assert np.array_equal(got, ref), (I, d)


@pytest.mark.parametrize("prec", [64, 32])
def test_c3_solve_residuals_consistent(c3, prec):
    import scipy.sparse as sp
    import torch
    p, S = c3
    S.set_precision(prec)
    u = S.solve(torch.tensor(p.f, device="cuda"))
    st = S.last_stats
    assert st["iterations"] == 60 or st["status"] == 0
    K = sp.bsr_matrix((p.vals, p.col, p.row_ptr.astype(np.int64)), shape=(p.n_dof, p.n_dof)).tocsr()
    rel = np.linalg.norm(p.f - K @ u.cpu().numpy()) / np.linalg.norm(p.f)
    assert abs(rel - st["relres_true"]) <= 1e-6 * max(rel, 1e-12)
    assert abs(st["relres_recursive"] - st["relres_true"]) <= 1e-3 * st["relres_true"]
