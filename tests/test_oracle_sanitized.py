"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a plain C
driver (oracle/sanitize_driver.c) runs its setup, a V-cycle and PCG on the
7^3 elasticity cube (six rigid-body modes) and on a random-modulus cube with the
paper's SRQCG test space, both built with -fsanitize=address,undefined.  The
run must end normally with no sanitizer report.  (The library's host code is
interleaved with device calls and cannot run without a GPU.)"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1902_01715_amd import problems as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def write_input(path, p, V0):
    n = p.n_nodes
    with open(path, "wb") as fh:
        fh.write(np.int32(n).tobytes())
        fh.write(np.int64(p.row_ptr[-1]).tobytes())
        fh.write(np.int32(V0.shape[-1]).tobytes())
        fh.write(np.asarray(p.row_ptr, dtype=np.int64).tobytes())
        fh.write(np.asarray(p.col, dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(p.vals, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(V0, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(p.f, dtype=np.float64).tobytes())


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", exe, os.path.join(ORACLE, "sanitize_driver.c"), "-lm"])
    return exe, d


def test_oracle_is_clean_under_sanitizers(sanitized_driver):
    exe, d = sanitized_driver
    rng = np.random.default_rng(9)
    cases = [("cube7", PR.c1_cube(7), None, 0)]
    q = PR.box_problem("r", 6, 6, 6, 1, 1, 1, E=10 ** rng.uniform(-2, 2, 216), nu=0.3, clamp="z0",
                       load=("body", (0, 0, -1)))
    cases.append(("randE6", q, PR.initial_test_space(q, 10, 11), 10))
    for name, p, V0, n_rq in cases:
        inp = str(d / f"{name}.bin")
        write_input(inp, p, p.V0 if V0 is None else V0)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe, inp, str(n_rq)], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, f"{name}: rc {r.returncode}\n{r.stdout}\n{r.stderr[-4000:]}"
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert "status 0" in r.stdout, r.stdout
