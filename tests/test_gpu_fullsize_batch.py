"""The multi-load-case workload at full size (cube 96^3, 2,738,019 DOF, 32
right-hand sides), in the configuration the benchmark times: the FP32 and the
FP64 cycle through solve_batch with the tuned tile.  Properties that hold at
any size: every column converges with a consistent true residual, and sampled
columns equal the single-right-hand-side solves of the same hierarchy."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4(cuda):
    from paper_1902_01715_amd import aspamg
    print("[case c4 full size, 32 load cases]", flush=True)
    p = PR.c4_multiload()
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0)
    yield p, S
    S.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_c4_batch_columns(c4, prec):
    import torch
    p, S = c4
    S.set_precision(prec)
    F = torch.tensor(p.f, device="cuda")
    U = S.solve_batch(F)
    stats = S.last_stats
    assert len(stats) == 32
    for j, st in enumerate(stats):
        assert st["status"] == 0, (j, st)
        assert st["relres_recursive"] <= 1e-10 and st["relres_true"] <= 2e-10, (j, st)
    assert stats[0]["spmm_tile"] in (4, 8, 16, 32)
    for j in (0, 17, 31):
        u1 = S.solve(F[:, j].contiguous())
        err = float(torch.linalg.norm(U[:, j] - u1) / torch.linalg.norm(u1))
        print(f"prec={prec} column {j}: it={stats[j]['iterations']} err vs single solve {err:.2e}")
        assert err <= 1e-8, (j, err)
