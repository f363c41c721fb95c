"""Failure handling of the oracle, forced from the host on the CPU: a NaN load,
a non-SPD matrix, the iteration cap and a zero load."""
import numpy as np
import pytest

import oracle as O
from paper_1902_01715_amd import problems as PR


@pytest.fixture(scope="module")
def cube(oracle_lib):
    p = PR.c1_cube(7)
    return p, O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)


def test_nan_load(cube):
    p, H = cube
    f = p.f.copy()
    f[5] = np.nan
    u, st = H.pcg(f, 1e-10, 100)
    assert st["status"] == O.ENAN


def test_iteration_cap(cube):
    p, H = cube
    u, st = H.pcg(p.f, 1e-10, 3)
    assert st["status"] == O.NOT_CONVERGED and st["iterations"] == 3 and st["relres"] > 1e-10


def test_zero_load(cube):
    p, H = cube
    u, st = H.pcg(np.zeros_like(p.f), 1e-10, 100)
    assert st["status"] == O.OK and st["iterations"] == 0 and not u.any()


def test_non_spd_matrix_is_rejected(oracle_lib):
    p = PR.c1_cube(7)
    vals = p.vals.copy()
    i = 200
    k = np.nonzero(p.col[p.row_ptr[i]:p.row_ptr[i + 1]] == i)[0][0] + p.row_ptr[i]
    vals[k] = -vals[k]
    with pytest.raises(RuntimeError, match="not SPD"):
        O.Hierarchy(p.row_ptr, p.col, vals, p.V0)


@pytest.fixture(scope="module")
def cantilever(oracle_lib):
    return PR.c2_cantilever(40, 4, 4)


def test_damping_beyond_two_over_lambda_breaks_pcg(cantilever):
    """Section 3.2: with omega lambda_1(G A G^T) > 2 the smoother diverges on
    the top of the spectrum and the V-cycle is no longer SPD.  The cantilever's
    fine level has lambda_1 = 2.44; a safety factor below 1 lets the applied
    omega reach min(1, .) = 1 and PCG must report a breakdown."""
    p = cantilever
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0, O.default_params(omega_safety=0.6))
    i0 = H.info(0)
    assert i0["omega_s"] * i0["lambda1"] > 2.0
    u, st = H.pcg(p.f, 1e-10, 1000)
    assert st["status"] == O.EBREAK, st
    # the default margin keeps omega lambda_1 below 2 and the solve converges
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    i0 = H.info(0)
    assert i0["omega_s"] * i0["lambda1"] < 2.0
    assert H.pcg(p.f, 1e-10, 1000)[1]["status"] == O.OK


def test_singular_matrix_is_rejected(oracle_lib):
    """No Dirichlet rows: K of a free body is singular (the rigid-body modes
    span its kernel), so the Galerkin operators are singular down to the
    coarsest level, whose Cholesky factorisation must refuse it."""
    q = PR.unconstrained_box(5, 5, 5, seed=1)
    with pytest.raises(RuntimeError, match="coarsest matrix not SPD"):
        O.Hierarchy(q.row_ptr, q.col, q.vals, q.V0)


def test_kappa_one_still_converges(cantilever):
    """kappa_p = 1 rejects every second interpolation column (and many first
    ones): P is very sparse, but the V-cycle stays an SPD preconditioner and
    PCG still converges, only slowly."""
    p = cantilever
    H0 = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0)
    H = O.Hierarchy(p.row_ptr, p.col, p.vals, p.V0, O.default_params(kappa_p=1.0))
    assert H.info(0)["nnzb_P"] < H0.info(0)["nnzb_P"]
    u, st = H.pcg(p.f, 1e-10, 5000)
    assert st["status"] == O.OK and st["iterations"] > H0.pcg(p.f, 1e-10, 1000)[1]["iterations"]
