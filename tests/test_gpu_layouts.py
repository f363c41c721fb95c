"""Both device layouts of the stored operators (sliced ELL with L lanes per row
and row-packed with K slot groups per lane in units of four wavefronts, where a
row's lanes may lie in different wavefronts), forced through the `layout`
parameter: every operator of every level against the oracle's matrices, the
solve against the oracle, and the slot-count policy giving the same layouts and
bitwise the same solution on two setups.  A randomly renumbered mesh, whose
slices span more than 65,536 columns, checks the 32-bit column fallback."""
import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

pytestmark = pytest.mark.gpu

POLICY = {"sliced": 2, "packed": 3, "packed64": 4}     # row-packed in workgroup / wavefront units


@pytest.fixture(scope="module")
def problem(oracle_lib):
    p = PR.c3_layered_distorted(32, 32, 16)   # 55,539 DOF, 4 levels, 68 PCG iterations
    H = oracle_lib.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    return p, H


@pytest.mark.parametrize("form", list(POLICY))
def test_forced_layout_operators_and_solve(cuda, problem, form, product_bound):
    import torch
    from paper_1902_01715_amd import aspamg
    p, H = problem
    print(f"[case layout {form}]", flush=True)
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(layout=POLICY[form]))
    assert S.nlev == H.nlev and S.nlev >= 3
    rng = np.random.default_rng(11)
    for l in range(H.nlev - 1):
        li = S.level_info(l)
        if li["sell_stacked"] != 0:     # 0: P, then A (A P denser than A)
            assert (li["sell_stacked"] > 0) == (form == "sliced")
        if form != "sliced" and li["sell_stacked"] != 0:   # the seam between P and A P starts a unit
            assert li["sell_index16"] & (1 << 10)
            assert li["sell_stacked_unit64"] == li["sell_stacked_unit32"] == (256 if form == "packed" else 64)
        for prec, lanes, units in ((64, li["sell_lanes64"], li["sell_unit64"]),
                                   (32, li["sell_lanes32"], li["sell_unit32"])):
            for which in range(5):
                fixed = l == 0 and which == 0     # q = K p copy (and its FP32 twin): sliced, one lane
                if fixed:
                    assert lanes[which] == 1 and units[which] == 0
                elif form == "sliced":
                    assert lanes[which] > 0 and units[which] == 0, (l, which, prec)
                else:
                    assert lanes[which] < 0, (l, which, prec)
                    assert units[which] == (256 if form == "packed" else 64), (l, which, prec)
                M = {0: H.A(l), 1: H.G(l), 2: H.G(l), 3: H.P(l), 4: H.P(l)}[which].to_scipy().tocsr()
                if which in (2, 4):
                    M = M.T.tocsr()
                x = rng.standard_normal(M.shape[1])
                y = S.apply(l, which, torch.tensor(x, device="cuda"), precision=prec,
                            out_rows=M.shape[0]).cpu().numpy()
                # FP64: the oracle's matrices differ from the device's by setup rounding
                bound = 1e-14 * (abs(M) @ np.abs(x)) + 1e-300 if prec == 64 else product_bound(M, x, 32)
                assert np.all(np.abs(y - M @ x) <= bound), (l, which, prec)
    for prec in (64, 32):
        S.set_precision(prec)
        u = S.solve(torch.tensor(p.f, device="cuda"), check=False).cpu().numpy()
        uo, sto = H.pcg(p.f, 1e-10, 1000)
        st = S.last_stats
        assert st["status"] == 0 and sto["status"] == 0
        # E = 1 / 1e4 layers: the recursive residual drifts from the true one in
        # both implementations, so the true residual is held to the oracle's own
        K = p.to_scipy().tocsr()
        rt_o = np.linalg.norm(p.f - K @ uo) / np.linalg.norm(p.f)
        err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
        print(f"{form} prec={prec} it={st['iterations']} (oracle {sto['iterations']}) err={err:.2e} "
              f"true res {st['relres_true']:.2e} (oracle {rt_o:.2e})", flush=True)
        assert st["relres_true"] <= 10 * max(rt_o, 1e-10)
        assert err <= 1e-8, err
    S.close()


def _crossing_rows(lens, K):
    """Rows whose lanes straddle a wavefront boundary inside a 256-lane unit of
    the row-packed plan (rows in order, max(1, ceil(len / K)) lanes each, a new
    unit when a row does not fit; no column-span break below 65,536 columns)."""
    used, cross = 256, 0
    for n in lens:
        lr = max(1, -(-int(n) // K))
        if used + lr > 256:
            used = 0
        cross += used // 64 != (used + lr - 1) // 64
        used += lr
    return cross


def test_packed_rows_cross_wavefronts(cuda, problem):
    """The forced row-packed layout of the problem above has rows whose lanes
    lie in two wavefronts (their partial sums meet across the workgroup), so the
    operator checks of test_forced_layout_operators_and_solve cover them."""
    from paper_1902_01715_amd import aspamg
    p, _ = problem
    assert p.n_nodes < 65536                   # every unit's columns fit 16-bit offsets
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(layout=POLICY["packed"]))
    try:
        total = 0
        for l in range(S.nlev - 1):
            li = S.level_info(l)
            for which in (1, 3):               # G and P: row lengths from the level's matrices
                K = -li["sell_lanes64"][which]
                rp = S.level_matrix(l, which)[0]
                total += _crossing_rows(np.diff(rp), K)
        assert total > 0
    finally:
        S.close()


def test_slot_policy_is_reproducible(cuda, problem):
    import torch
    from paper_1902_01715_amd import aspamg
    p, _ = problem
    outs, lays = [], []
    for _ in range(2):
        S = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, aspamg.default_params(layout=1))
        lays.append([(S.level_info(l)["sell_lanes64"], S.level_info(l)["sell_lanes32"], S.level_info(l)["sell_stacked"])
                     for l in range(S.nlev)])
        S.set_precision(32)
        outs.append(S.solve(torch.tensor(p.f, device="cuda"), check=False).cpu().numpy())
        S.close()
    assert lays[0] == lays[1]
    assert np.array_equal(outs[0], outs[1])


def _permuted(p, seed):
    """The problem with its nodes renumbered by a random permutation."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n = p.n_nodes
    perm = rng.permutation(n)                 # old node -> new node
    inv = np.argsort(perm)
    rp = np.asarray(p.row_ptr, dtype=np.int64)
    B = sp.bsr_matrix((p.vals, p.col, rp), shape=(3 * n, 3 * n)).tocsr()
    P = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    P3 = sp.kron(P, sp.identity(3), format="csr")
    Bp = (P3 @ B @ P3.T).tobsr(blocksize=(3, 3))
    Bp.sort_indices()
    V0 = np.ascontiguousarray(p.V0[inv])
    f = np.ascontiguousarray(p.f.reshape(n, 3)[inv].reshape(-1))
    return (Bp.indptr.astype(np.int32), Bp.indices.astype(np.int32), np.ascontiguousarray(Bp.data), V0, f, Bp.tocsr())


def test_wide_column_spans_use_32bit_indices(cuda, product_bound):
    import scipy.sparse as sp
    import torch
    from paper_1902_01715_amd import aspamg
    print("[case permuted cube 41^3]", flush=True)
    p = PR.c1_cube(41)                         # 74,088 nodes
    rp, ci, v, V0, f, K = _permuted(p, 5)
    S = aspamg.Solver(rp, ci, v, V0)
    li = S.level_info(0)
    # randomly numbered rows: a slice spans more than 65,536 columns
    assert not li["sell_index16"] & 1 and not li["sell_index16"] & (1 << 5)
    n, nc = li["n"], li["n_coarse"]
    r2, c2, v2 = S.level_matrix(0, 0)
    A = sp.bsr_matrix((v2, c2, r2), shape=(3 * n, 3 * n)).tocsr()
    r2, c2, v2 = S.level_matrix(0, 1)
    G = sp.bsr_matrix((v2, c2, r2), shape=(3 * n, 3 * n)).tocsr()
    r2, c2, v2 = S.level_matrix(0, 3)
    P = sp.bsr_matrix((v2, c2, r2), shape=(3 * n, 3 * nc)).tocsr()
    ops = [A, G, G.T.tocsr(), P, P.T.tocsr()]
    rng = np.random.default_rng(2)
    for prec in (64, 32):
        for which, M in enumerate(ops):
            x = rng.standard_normal(M.shape[1])
            y = S.apply(0, which, torch.tensor(x, device="cuda"), precision=prec, out_rows=M.shape[0]).cpu().numpy()
            assert np.all(np.abs(y - M @ x) <= product_bound(M, x, prec)), (which, prec)
    u = S.solve(torch.tensor(f, device="cuda")).cpu().numpy()
    assert S.last_stats["status"] == 0
    assert np.linalg.norm(f - K @ u) <= 2e-10 * np.linalg.norm(f)
    S.close()
