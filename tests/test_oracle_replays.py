"""Pins of the oracle's decision rules against independent replays and closed forms.

The aFSAI growth, its eps_g stop and outer loop (Section 3.1, Algorithm "aFSAI
Smoother Set-up"), the theta filter of the strong graph (Section 3.4) and the
interpolation candidates (Section 3.5) are each restated from the rule in
`oracle_replay.py` with numpy/scipy arithmetic and compared with what the
oracle decides.  `test_oracle_mutations.py` plants plausible mistakes in copies
of the oracle and checks that these pins catch each one."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import oracle_replay as RP
from paper_1902_01715_amd import problems as PR


def tridiagonal(n, diag=2.0, off=-1.0):
    """b = 1 tridiagonal (diag, off) in the oracle's BSR input form."""
    A = sp.diags([np.full(n - 1, off), np.full(n, diag), np.full(n - 1, off)], [-1, 0, 1], format="csr")
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.reshape(-1, 1, 1).copy(), A


def random_cube(n=7, seed=11, jitter=0.3):
    """Jittered cube with E = 10^U[-2,2] per element: no two candidates tie."""
    rng = np.random.default_rng(seed)
    E = 10.0 ** rng.uniform(-2, 2, n ** 3)
    return PR.box_problem(f"rc{n}", n, n, n, 1.0, 1.0, 1.0, E=E, nu=0.3, clamp="z0",
                          load=("body", (0, 0, -1)), jitter=jitter, rng=rng)


# ----------------------------------------------------------------------------- aFSAI growth: closed forms
def test_growth_on_tridiagonal_adds_next_lower_neighbour(oracle_lib):
    """b = 1 tridiagonal: the only candidate of row I below I and outside B is
    the next lower node, so k steps give B = {I-k, ..., I-1} (fewer near row 0).
    For the (2, -1) matrix the local system of a window of m + 1 entries is the
    leading block of the 1D Laplacian, whose last Schur complement is
    psi = (m + 2) / (m + 1)."""
    n = 40
    rp, ci, v, A = tridiagonal(n)
    rows = np.array([0, 1, 2, 5, 17, 39], dtype=np.int32)
    for k_g in (1, 2, 3, 4):
        prm = O.default_params(b=1, k_g=k_g, rho_b=3, eps_g=0.0)
        pats, g, psi = O.fsai_rows(prm, rp, ci, v, rows)
        for r, I in enumerate(rows):
            m = min(k_g, int(I))
            assert list(pats[r]) == list(range(I - m, I))
            assert abs(psi[r, 0] - (m + 2) / (m + 1)) <= 1e-14
            # the stored row is the inverse-Cholesky row of the window
            win = list(range(I - m, I + 1))
            Lw = np.linalg.cholesky(A[win][:, win].toarray())
            assert np.allclose(g[r, 0, :m + 1], np.linalg.inv(Lw)[-1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("eps,expect_nb", [
    (1.0 / 16.0, 3),                          # q(psi_prev - psi) == q(eps psi_prev) at the third step: stop
    (1.0 / 16.0 * (1.0 - 2.0 ** -30), 3),     # below the quantum: still equal after rounding, stop
    (1.0 / 16.0 * (1.0 - 2.0 ** -12), 4),     # a resolved margin: the third step continues
    (1.0 / 4.0, 1),                           # relative decrease 1/4 at the first step: stop there
    (0.0, 4),                                 # eps_g = 0: only k_g ends the pass
])
def test_eps_stop_fires_exactly_at_threshold(eps, expect_nb, oracle_lib):
    """On the (2, -1) tridiagonal, growing from |B| = j to j + 1 lowers psi from
    (j+2)/(j+1) to (j+3)/(j+2), a relative decrease of exactly 1/(j+2)^2.  The
    row stops once q(psi_prev - psi) <= q(eps_g psi_prev) (R-F5, decision values
    rounded to 20 bits): with eps_g = 1/16 that is the step to |B| = 3."""
    n = 30
    rp, ci, v, _ = tridiagonal(n)
    prm = O.default_params(b=1, k_g=4, rho_b=3, eps_g=eps)
    pats, _, _ = O.fsai_rows(prm, rp, ci, v, np.array([20], dtype=np.int32))
    assert len(pats[0]) == expect_nb


# ----------------------------------------------------------------------------- aFSAI growth: replay
@pytest.fixture(scope="module")
def rcube(oracle_lib):
    p = random_cube()
    A = p.to_scipy().toarray()
    adj = RP.node_adjacency(p.row_ptr, p.col)
    return p, A, adj


def test_growth_steps_replay(rcube):
    """Sampled rows of a jittered random-E cube: after 1..4 growth steps the
    oracle's pattern equals the replay's (gradient h = A g' on the candidates
    adjacent to B u {I}, the rho_b = 3 largest quantised scores), and its psi
    equals the local minimum of g^T A g."""
    p, A, adj = rcube
    rng = np.random.default_rng(3)
    free = np.nonzero(~p.dirichlet)[0]
    rows = np.sort(rng.choice(free[free > 60], 40, replace=False)).astype(np.int32)
    for k_g in (1, 2, 3, 4):
        prm = O.default_params(k_g=k_g, eps_g=0.0)
        pats, _, psi = O.fsai_rows(prm, O.problem_rp(p), p.col, p.vals, rows)
        for r, I in enumerate(rows):
            ref = RP.first_pass(A, adj, int(I), k_g, 3, 0.0)
            assert list(pats[r]) == ref, (k_g, I)
            _, psi_ref, _ = RP.fsai_row(A, int(I), ref)
            assert np.allclose(psi[r], psi_ref, rtol=1e-12)


def test_first_pass_replay_with_eps_stop(rcube):
    """The default first pass (k_g = 4, eps_g = 1e-3) and a coarse eps_g = 0.05,
    where most rows stop early, on every free row of the cube's upper half."""
    p, A, adj = rcube
    rows = np.array([i for i in range(p.n_nodes // 2, p.n_nodes) if not p.dirichlet[i]], dtype=np.int32)
    for eps in (1e-3, 0.05):
        prm = O.default_params(eps_g=eps)
        pats, _, _ = O.fsai_rows(prm, O.problem_rp(p), p.col, p.vals, rows)
        lens = []
        for r, I in enumerate(rows):
            ref = RP.first_pass(A, adj, int(I), 4, 3, eps)
            assert list(pats[r]) == ref, (eps, I)
            lens.append(len(ref))
        if eps == 0.05:
            assert min(lens) < 12 and max(lens) == 12          # the stop fires on some rows, not all


@pytest.mark.parametrize("n,stop", [(6, "density"), (5, "omega")])
def test_outer_loop_replay(n, stop, oracle_lib):
    """A first-pass G on these cubes gives omega_q = 2/lambda_1 of about 1.13,
    so omega_bar = 1.2 makes the outer loop grow every row by one step per
    round: on the 6^3 cube until G holds as many blocks as A (density stop), on
    the 5^3 cube until omega_q passes 1.2.  The replay (dense lambda_1) takes
    the same rounds to the same stop and gives the same patterns."""
    p = random_cube(n, seed=12)
    A = p.to_scipy().toarray()
    adj = RP.node_adjacency(p.row_ptr, p.col)
    prm = O.default_params(omega_bar=1.2, coarse_max_dof=300)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0, prm)
    assert H.nlev >= 2
    info = H.info(0)
    G = H.G(0)
    pats, rounds, hist = RP.outer_loop(A, adj, p.nnzb, 4, 3, 1e-3, 1.2)
    assert info["fsai_rounds"] == rounds >= 2
    assert all(w < 1.2 for _, w in hist[:-1]) and all(nb < p.nnzb for nb, _ in hist[:-1])
    if stop == "density":
        assert hist[-1][0] >= p.nnzb and hist[-1][1] < 1.2
    else:
        assert hist[-1][0] < p.nnzb and hist[-1][1] >= 1.2
    assert abs(info["omega_q"] - hist[-1][1]) <= 2e-3 * hist[-1][1]
    for I in range(p.n_nodes):
        assert list(G.ci[G.rp[I]:G.rp[I + 1] - 1]) == pats[I], I
    # omega_bar below the first pass's omega_q: no extra round
    H2 = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0,
                     O.default_params(omega_bar=hist[0][1] * 0.999, coarse_max_dof=300))
    assert H2.info(0)["fsai_rounds"] == 0


# ----------------------------------------------------------------------------- theta filter, candidates
@pytest.fixture(scope="module")
def srq_hier(oracle_lib):
    """A hierarchy whose test space is smoothed by SRQCG, so SoC values spread out."""
    p = random_cube(7, seed=13)
    V0 = PR.initial_test_space(p, 10, 7)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, V0, O.default_params(n_rq=4))
    return p, H


@pytest.mark.parametrize("which", ["c1", "srq"])
def test_theta_filter_replay(which, srq_hier, c1_hier):
    """S equals min(theta, deg) strongest SoC > 0 per node (quantised, ties to
    the lowest J), symmetrised by union; SoC equals the node affinity of the
    level's test space."""
    p, H = srq_hier if which == "srq" else c1_hier
    for l in range(H.nlev - 1):
        A = H.A(l)
        rp, ci = A.rp, A.ci
        excl = np.array([rp[i + 1] - rp[i] == 1 for i in range(A.n)])
        soc = H.soc(l)
        ref_soc = RP.soc_from_V(H.V(l), rp, ci, excl)
        assert np.allclose(soc, ref_soc, rtol=1e-12, atol=1e-15)
        srp, sci = H.S(l)
        S = RP.theta_filter(rp, ci, soc, H.p.theta)
        for i in range(A.n):
            assert set(sci[srp[i]:srp[i + 1]]) == S[i], (l, i)


@pytest.fixture(scope="module")
def c1_hier(oracle_lib):
    p = PR.c1_cube(10)
    return p, O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)


@pytest.mark.parametrize("which", ["c1", "srq"])
def test_interpolation_candidates_replay(which, srq_hier, c1_hier):
    """Each F node's candidates are the C nodes at S-distance 1..d_p (scipy
    shortest paths), and every chosen interpolation column is one of them."""
    p, H = srq_hier if which == "srq" else c1_hier
    for l in range(H.nlev - 1):
        cf = H.cf(l)
        srp, sci = H.S(l)
        ref = RP.candidates_within(srp, sci, cf, H.p.d_p)
        crp, cci = H.candidates(l)
        cidx = np.cumsum(cf == 1) - 1
        cnt, cols = H.P_scalar(l)
        far = 0
        for i in range(len(cf)):
            got = list(cci[crp[i]:crp[i + 1]])
            assert got == ref.get(i, []), (l, i)
            if cf[i] == 0:
                Cset = {int(cidx[j]) for j in got}
                for d in range(3):
                    for k in range(cnt[3 * i + d]):
                        assert cols[3 * i + d, k] // 3 in Cset
        # depth 2 matters: some rows use a C node that is not an S-neighbour
        for i in np.nonzero(cf == 0)[0]:
            nb = set(sci[srp[i]:srp[i + 1]])
            used = {int(np.nonzero(cidx == c)[0][0]) for d in range(3) for c in cols[3 * i + d, :cnt[3 * i + d]] // 3}
            far += bool(used - nb)
        if l == 0:
            assert far > 0
