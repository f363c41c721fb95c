import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libaspamg.so")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1902_01715_amd import aspamg
    aspamg.lib()          # fails loudly when the library is missing
    return torch.device("cuda:0")


def _product_bound(M, x, prec):
    """Per-row bound on |y - M x|, y the device product in IEEE precision `prec`
    (64 or 32) and M x the host reference in FP64.  Rounding the entries of M
    and x to `prec` and summing each row in that precision, in any order, errs by
    at most gamma_{m+2} |M| |x| (gamma_m for FP64, whose operands are exact),
    m the row's stored entries and gamma_k = k u / (1 - k u) (Higham, Accuracy
    and Stability of Numerical Algorithms, 2nd ed., Sec. 3.1); the FP64
    reference adds its own gamma_m.  A factor 1.25 covers the rounding of the
    bound's evaluation."""
    import numpy as np
    m = M.getnnz(axis=1).astype(np.float64)
    gamma = lambda k, u: k * u / (1 - k * u)
    u64 = 2.0 ** -53
    g = gamma(m, u64) + (gamma(m, u64) if prec == 64 else gamma(m + 2, 2.0 ** -24))
    return 1.25 * g * (abs(M) @ np.abs(x)) + 1e-300


@pytest.fixture(scope="session")
def product_bound():
    return _product_bound
