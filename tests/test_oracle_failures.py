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
