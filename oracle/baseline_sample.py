"""TEST INFRASTRUCTURE: the bounded sample on which the CPU baseline of the
benchmark times the oracle, and the OpenMP timing build it uses.

A sample is a small instance of the benchmark workload's own recipe (same
element size, materials, test space and parameters): the layered block
32x32x16 for the layered workload, the 20x32x32 leading slab for the
cantilever, 20^3 tetrahedra for the scalar workload.  time_sample() builds the oracle's hierarchy for it and times a
fixed number of PCG iterations on one thread and on all host cores.  The same
function runs on the host where oracle/fullsize_run.py measured the full-size
workload, so the ratio between the two hosts scales that measurement.
"""
from __future__ import annotations

import os
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
_OMP_LIB = None


def openmp_build():
    """Compile the OpenMP timing build of the oracle once per process."""
    global _OMP_LIB
    if _OMP_LIB is None:
        import oracle
        d = tempfile.mkdtemp(prefix="oracle_omp_")
        _OMP_LIB = oracle.compile_source(os.path.join(HERE, "aspamg_oracle.c"), os.path.join(d, "liboracle_omp.so"),
                                         openmp=True)
    return _OMP_LIB


def host_threads():
    """Threads the host offers: OMP_NUM_THREADS when set, else the CPU count."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def sample_problem(config):
    from paper_1902_01715_amd import problems as PR
    if config == "c3":
        return PR.c3_layered_distorted(32, 32, 16), "layered block 32x32x16 (55,539 DOF), the C3 recipe"
    if config == "c2":
        return PR.c2_cantilever(20, 32, 32), "20x32x32 leading slab of the cantilever (68,607 DOF)"
    if config == "t1":
        return PR.tet_elasticity(20, 20, 20, jitter=0.2, seed=6), \
            "point-wise elasticity on 20^3 x 6 tetrahedra (27,783 unknowns), the t1 recipe"
    raise ValueError(config)


def time_sample(config, n_rq, iters=20):
    """{'desc', 'n_dof', 'setup_s', 'pcg': {threads: s_per_iter}} of the sample."""
    import oracle
    from paper_1902_01715_amd import problems as PR
    oracle.use_library(openmp_build())
    p, desc = sample_problem(config)
    V0 = p.V0 if n_rq == 0 else PR.initial_test_space(p, 10, 11)
    nt = host_threads()
    oracle.set_threads(nt)
    t0 = time.perf_counter()
    from oracle.fullsize_run import scalar_params
    H = oracle.Hierarchy(p.row_ptr, p.col, p.vals, V0, oracle.default_params(n_rq=n_rq, **scalar_params(config)))
    setup = time.perf_counter() - t0
    out = {"desc": desc, "n_dof": int(p.n_dof), "setup_s": setup, "iterations": iters, "pcg": {}}
    for threads in sorted({1, nt}):
        got = oracle.set_threads(threads)
        H.pcg(p.f, 0.0, 1)
        t0 = time.perf_counter()
        _, st = H.pcg(p.f, 0.0, iters)
        out["pcg"][str(got)] = (time.perf_counter() - t0) / st["iterations"]
    del H
    oracle.use_library(None)
    return out
