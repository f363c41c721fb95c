"""TEST INFRASTRUCTURE: ctypes wrapper of the plain FP64 CPU oracle (aspamg_oracle.c).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aspamg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, ENOTSPD, EBREAK, ENAN = 0, 1, -1, -2, -4, -5, -6


def compile_source(src: str, out: str, openmp: bool = False) -> str:
    """gcc build of one oracle source file (no fast-math, no FP contraction);
    openmp=True builds the timing variant whose row loops run on all cores."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
                          + (["-fopenmp"] if openmp else []) + ["-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("b", C.c_int32), ("k_g", C.c_int32), ("rho_b", C.c_int32), ("eps_g", C.c_double),
        ("theta", C.c_int32), ("n_max", C.c_int32), ("kappa_p", C.c_double),
        ("omega_bar", C.c_double), ("outer_fsai", C.c_int32), ("d_p", C.c_int32),
        ("eps_p", C.c_double), ("lanczos_steps", C.c_int32), ("omega_safety", C.c_double),
        ("coarse_max_dof", C.c_int32), ("max_levels", C.c_int32), ("stall_ratio", C.c_double),
        ("nu1", C.c_int32), ("nu2", C.c_int32), ("quant_bits", C.c_int32),
        ("dense_max_dof", C.c_int32), ("n_rq", C.c_int32), ("k_ritz", C.c_int32),
    ]


_lib = None
# None: the built liboracle.so; else another compiled copy of the source (see
# use_library; ORACLE_LIBRARY in the environment sets it for a whole process)
_lib_path = os.environ.get("ORACLE_LIBRARY") or None


def use_library(path):
    """Load the oracle from another compiled copy of its source (or, with None,
    the built one again).  The mutation tests use it to run the pins against
    copies with a planted mistake."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        path = _lib_path
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        P = C.c_void_p
        L.oracle_setup.restype = C.c_int
        L.oracle_setup.argtypes = [C.POINTER(Params), C.c_int32, P, P, P, C.c_int32, P, C.POINTER(C.c_void_p)]
        L.oracle_free.argtypes = [C.c_void_p]
        L.oracle_num_levels.argtypes = [C.c_void_p]
        L.oracle_min_margin.argtypes = [C.c_void_p]
        L.oracle_min_margin.restype = C.c_double
        L.oracle_coarse_order.argtypes = [C.c_void_p]
        L.oracle_level_info.argtypes = [C.c_void_p, C.c_int, P, P]
        for nm in ("oracle_level_A", "oracle_level_G", "oracle_level_P"):
            getattr(L, nm).argtypes = [C.c_void_p, C.c_int, P, P, P]
        L.oracle_level_cf.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_level_V.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_level_S.argtypes = [C.c_void_p, C.c_int, P, P]
        L.oracle_level_soc.argtypes = [C.c_void_p, C.c_int, P]
        L.oracle_level_Pscalar.argtypes = [C.c_void_p, C.c_int, P, P]
        L.oracle_level_candidates.restype = C.c_int64
        L.oracle_level_candidates.argtypes = [C.c_void_p, C.c_int, P, P]
        L.oracle_coarse_factor.argtypes = [C.c_void_p, P]
        L.oracle_vcycle.argtypes = [C.c_void_p, P, P]
        L.oracle_pcg.restype = C.c_int
        L.oracle_pcg.argtypes = [C.c_void_p, P, P, C.c_double, C.c_int, P, P]
        L.oracle_element_gradient.argtypes = [C.c_int64, P, P, C.c_int64, P, P, P]
        L.oracle_fsai_fixed.restype = C.c_int
        L.oracle_fsai_fixed.argtypes = [C.c_int32, C.c_int, P, P, P, P, P, P, P, P, P]
        L.oracle_fsai_rows.restype = C.c_int
        L.oracle_fsai_rows.argtypes = [C.POINTER(Params), C.c_int32, P, P, P, C.c_int32, P, P, P, P, P]
        L.oracle_lanczos.restype = C.c_double
        L.oracle_lanczos.argtypes = [C.c_int32, C.c_int, P, P, P, P, P, P, C.c_int]
        L.oracle_srqcg.restype = C.c_int
        L.oracle_srqcg.argtypes = [C.c_int32, C.c_int, P, P, P, P, P, P, C.c_int, P, C.c_int, C.c_int, P]
        L.oracle_dpls_row.restype = C.c_int
        L.oracle_dpls_row.argtypes = [C.POINTER(Params), P, P, C.c_int, C.c_int, P, P]
        L.oracle_rap.restype = C.c_int
        L.oracle_rap.argtypes = [C.c_int32, C.c_int32, C.c_int, P, P, P, P, P, P, P, P, P, P, C.c_int64]
        L.oracle_soc_node.restype = C.c_double
        L.oracle_soc_node.argtypes = [P, C.c_int, C.c_int, C.c_int32, C.c_int32]
        L.oracle_mis.argtypes = [C.c_int32, P, P, P, P]
        L.oracle_orthonormalize.argtypes = [P, C.c_int64, C.c_int]
        L.oracle_quantize.restype = C.c_double
        L.oracle_quantize.argtypes = [C.c_double, C.c_int]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64]
        L.oracle_last_error.restype = C.c_char_p
        L.oracle_default_params.argtypes = [C.POINTER(Params)]
        L.oracle_max_nb.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def default_params(**kw) -> Params:
    p = Params()
    lib().oracle_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class BSR:
    """Plain BSR container: rp int64 [n+1], ci int32, v float64 [nnzb, b, b]."""

    def __init__(self, rp, ci, v, n, nc, b):
        self.rp, self.ci, self.v, self.n, self.nc, self.b = rp, ci, v, n, nc, b

    @property
    def nnzb(self):
        return int(self.rp[-1])

    def to_dense(self):
        b = self.b
        D = np.zeros((self.n * b, self.nc * b))
        for i in range(self.n):
            for k in range(self.rp[i], self.rp[i + 1]):
                j = self.ci[k]
                D[i * b:(i + 1) * b, j * b:(j + 1) * b] = self.v[k]
        return D

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bsr_matrix((self.v, self.ci, self.rp), shape=(self.n * self.b, self.nc * self.b))


def _bsr_args(rp, ci, v):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return rp, ci, v


class Hierarchy:
    """The oracle's aSP-AMG hierarchy for an SPD BSR matrix and test space V0."""

    def __init__(self, rp, ci, v, V0, params: Params | None = None, b: int = 3):
        self.p = params if params is not None else default_params(b=b)
        self.b = self.p.b
        rp, ci, v = _bsr_args(rp, ci, v)
        self.n = rp.shape[0] - 1
        V0 = np.ascontiguousarray(V0, dtype=np.float64)
        self.ntv = V0.shape[-1] if V0.size else 0
        h = C.c_void_p()
        rc = lib().oracle_setup(C.byref(self.p), self.n, _p(rp), _p(ci), _p(v), self.ntv, _p(V0), C.byref(h))
        if rc < 0:
            raise RuntimeError(f"oracle setup failed ({rc}): {lib().oracle_last_error().decode()}")
        self.h = h
        self._keep = (rp, ci, v)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_free(h)
            self.h = None

    @property
    def nlev(self):
        return lib().oracle_num_levels(self.h)

    @property
    def min_margin(self):
        return lib().oracle_min_margin(self.h)

    def info(self, l):
        i = np.zeros(10, dtype=np.int64)
        d = np.zeros(4)
        lib().oracle_level_info(self.h, l, _p(i), _p(d))
        return dict(n=int(i[0]), nnzb_A=int(i[1]), nnzb_G=int(i[2]), nnzb_P=int(i[3]), nc=int(i[4]),
                    fsai_rounds=int(i[5]), has_G=bool(i[6]), has_P=bool(i[7]), nnz_S=int(i[8]),
                    lambda1=d[0], omega_q=d[1], omega_s=d[2])

    def _get(self, fn, l, n, nc, nnzb):
        b = self.b
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(max(nnzb, 1), dtype=np.int32)
        v = np.zeros((max(nnzb, 1), b, b))
        fn(self.h, l, _p(rp), _p(ci), _p(v))
        return BSR(rp, ci[:nnzb], v[:nnzb], n, nc, b)

    def A(self, l):
        i = self.info(l)
        return self._get(lib().oracle_level_A, l, i["n"], i["n"], i["nnzb_A"])

    def G(self, l):
        i = self.info(l)
        return self._get(lib().oracle_level_G, l, i["n"], i["n"], i["nnzb_G"])

    def P(self, l):
        i = self.info(l)
        return self._get(lib().oracle_level_P, l, i["n"], i["nc"], i["nnzb_P"])

    def cf(self, l):
        out = np.zeros(self.info(l)["n"], dtype=np.int8)
        lib().oracle_level_cf(self.h, l, _p(out))
        return out

    def V(self, l):
        n = self.info(l)["n"]
        out = np.zeros((n, self.b, self.ntv))
        lib().oracle_level_V(self.h, l, _p(out))
        return out

    def S(self, l):
        i = self.info(l)
        rp = np.zeros(i["n"] + 1, dtype=np.int64)
        ci = np.zeros(max(i["nnz_S"], 1), dtype=np.int32)
        lib().oracle_level_S(self.h, l, _p(rp), _p(ci))
        return rp, ci[:i["nnz_S"]]

    def soc(self, l):
        out = np.zeros(max(self.info(l)["nnzb_A"], 1))
        lib().oracle_level_soc(self.h, l, _p(out))
        return out

    def P_scalar(self, l):
        n = self.info(l)["n"]
        cnt = np.zeros(n * self.b, dtype=np.int32)
        cols = np.zeros((n * self.b, self.p.n_max), dtype=np.int32)
        lib().oracle_level_Pscalar(self.h, l, _p(cnt), _p(cols))
        return cnt, cols

    def candidates(self, l):
        """Interpolation candidates (C nodes within S-distance d_p) of each F node: (rp, ci)."""
        n = self.info(l)["n"]
        rp = np.zeros(n + 1, dtype=np.int64)
        tot = lib().oracle_level_candidates(self.h, l, _p(rp), None)
        ci = np.zeros(max(tot, 1), dtype=np.int32)
        lib().oracle_level_candidates(self.h, l, _p(rp), _p(ci))
        return rp, ci[:tot]

    def coarse_factor(self):
        nd = lib().oracle_coarse_order(self.h)
        L = np.zeros((nd, nd))
        lib().oracle_coarse_factor(self.h, _p(L))
        return L

    def vcycle(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        z = np.zeros_like(y)
        lib().oracle_vcycle(self.h, _p(y), _p(z))
        return z

    def pcg(self, f, rtol=1e-10, max_it=1000):
        f = np.ascontiguousarray(f, dtype=np.float64)
        u = np.zeros_like(f)
        it = np.zeros(1, dtype=np.int32)
        rr = np.zeros(1)
        rc = lib().oracle_pcg(self.h, _p(f), _p(u), rtol, max_it, _p(it), _p(rr))
        return u, dict(status=rc, iterations=int(it[0]), relres=float(rr[0]))

    def complexities(self):
        n0 = self.info(0)
        cgd = sum(self.info(l)["n"] for l in range(self.nlev)) / n0["n"]
        cop = sum(self.info(l)["nnzb_A"] for l in range(self.nlev)) / n0["nnzb_A"]
        return cgd, cop


def fsai_fixed(rp, ci, v, brp, bci, b=3):
    """FSAI factor for a prescribed pattern (B per block row); returns (G BSR, psi)."""
    rp, ci, v = _bsr_args(rp, ci, v)
    n = rp.shape[0] - 1
    brp = np.ascontiguousarray(brp, dtype=np.int64)
    bci = np.ascontiguousarray(bci, dtype=np.int32)
    grp = np.zeros(n + 1, dtype=np.int64)
    nnzg = int(brp[-1]) + n
    gci = np.zeros(nnzg, dtype=np.int32)
    gv = np.zeros((nnzg, b, b))
    psi = np.zeros(n * b)
    rc = lib().oracle_fsai_fixed(n, b, _p(rp), _p(ci), _p(v), _p(brp), _p(bci), _p(grp), _p(gci), _p(gv), _p(psi))
    if rc != 0:
        raise RuntimeError(f"fsai_fixed failed {rc}")
    return BSR(grp, gci, gv, n, n, b), psi


def fsai_rows(params, rp, ci, v, rows):
    """First adaptive FSAI pass for selected block rows: (patterns list, g, psi)."""
    rp, ci, v = _bsr_args(rp, ci, v)
    n = rp.shape[0] - 1
    b = params.b
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    mnb = lib().oracle_max_nb()
    nodes = np.zeros((rows.size, mnb), dtype=np.int32)
    nb = np.zeros(rows.size, dtype=np.int32)
    g = np.zeros((rows.size, b, mnb * b + b))
    psi = np.zeros((rows.size, b))
    rc = lib().oracle_fsai_rows(C.byref(params), n, _p(rp), _p(ci), _p(v), rows.size, _p(rows), _p(nodes),
                                _p(nb), _p(g), _p(psi))
    if rc != 0:
        raise RuntimeError(f"fsai_rows failed {rc}")
    return [nodes[r, :nb[r]].copy() for r in range(rows.size)], g, psi


def lanczos(rp, ci, v, G: BSR, steps=30, b=3):
    rp, ci, v = _bsr_args(rp, ci, v)
    n = rp.shape[0] - 1
    grp, gci, gv = _bsr_args(G.rp, G.ci, G.v)
    return lib().oracle_lanczos(n, b, _p(rp), _p(ci), _p(v), _p(grp), _p(gci), _p(gv), steps)


def srqcg(rp, ci, v, G: BSR, V0, kmax, kritz=1, b=3):
    """Test space by SRQCG on S = G A G^T; V0 [n*b, nt].  Returns (G^T Z, the
    final Rayleigh quotients of the columns of Z)."""
    rp, ci, v = _bsr_args(rp, ci, v)
    n = rp.shape[0] - 1
    grp, gci, gv = _bsr_args(G.rp, G.ci, G.v)
    V = np.array(V0, dtype=np.float64, order="C", copy=True).reshape(n * b, -1)
    nt = V.shape[1]
    rq = np.zeros(nt)
    rc = lib().oracle_srqcg(n, b, _p(rp), _p(ci), _p(v), _p(grp), _p(gci), _p(gv), nt, _p(V), kmax, kritz, _p(rq))
    if rc != 0:
        raise RuntimeError(f"srqcg failed {rc}")
    return V, rq


def dpls_row(params, v, Cm):
    v = np.ascontiguousarray(v, dtype=np.float64)
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    nca, ntv = Cm.shape
    chosen = np.zeros(16, dtype=np.int32)
    w = np.zeros(16)
    k = lib().oracle_dpls_row(C.byref(params), _p(v), _p(Cm), nca, ntv, _p(chosen), _p(w))
    if k < 0:
        raise RuntimeError(f"dpls_row failed ({k}): {lib().oracle_last_error().decode()}")
    return chosen[:k].copy(), w[:k].copy()


def rap(A: BSR, P: BSR):
    rp, ci, v = _bsr_args(A.rp, A.ci, A.v)
    prp, pci, pv = _bsr_args(P.rp, P.ci, P.v)
    b = A.b
    nnz = np.zeros(1, dtype=np.int64)
    cap = P.nc * P.nc
    crp = np.zeros(P.nc + 1, dtype=np.int64)
    cci = np.zeros(cap, dtype=np.int32)
    cv = np.zeros((cap, b, b))
    rc = lib().oracle_rap(A.n, P.nc, b, _p(rp), _p(ci), _p(v), _p(prp), _p(pci), _p(pv), _p(nnz), _p(crp),
                          _p(cci), _p(cv), cap)
    if rc != 0:
        raise RuntimeError(f"rap failed {rc}")
    k = int(nnz[0])
    return BSR(crp, cci[:k], cv[:k], P.nc, P.nc, b)


def soc_node(V, I, J):
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, b, ntv = V.shape
    return lib().oracle_soc_node(_p(V), b, ntv, I, J)


def mis(srp, sci, excluded=None):
    srp = np.ascontiguousarray(srp, dtype=np.int64)
    sci = np.ascontiguousarray(sci, dtype=np.int32)
    n = srp.shape[0] - 1
    cf = np.zeros(n, dtype=np.int8)
    ex = None if excluded is None else np.ascontiguousarray(excluded, dtype=np.int8)
    lib().oracle_mis(n, _p(srp), _p(sci), _p(ex), _p(cf))
    return cf


def orthonormalize(V):
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    ntv = V.shape[-1]
    lib().oracle_orthonormalize(_p(V), V.size // ntv, ntv)
    return V


def quantize(s, bits=20):
    return lib().oracle_quantize(float(s), bits)


def splitmix64(x):
    return lib().oracle_splitmix64(int(x))


def element_gradient(conn, Ke0, lam, u, ke_stride=0):
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    Ke0 = np.ascontiguousarray(Ke0, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n_el = conn.shape[0]
    g = np.zeros(n_el)
    lib().oracle_element_gradient(n_el, _p(conn), _p(Ke0), ke_stride, _p(lam), _p(u), _p(g))
    return g


def problem_rp(problem):
    """int64 row pointer of a Problem's K (the oracle's index width)."""
    return np.asarray(problem.row_ptr, dtype=np.int64)


def set_threads(n):
    """Threads of the OpenMP timing build (no effect on the default build)."""
    lib().oracle_set_threads(int(n))
    return lib().oracle_threads()
