"""Python binding of libaspamg.so (the aSP-AMG solve phase on MI355X).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the HIP stream.  The
binding fails loudly when the compiled library is missing; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaspamg.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENOT_SPD, EBREAKDOWN, ENAN = 0, 1, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOT_SPD",
                -5: "EBREAKDOWN", -6: "ENAN"}

# every symbol declared in include/aspamg.h
EXPORTED = [
    "aspamg_default_params", "aspamg_setup", "aspamg_set_cycle_precision", "aspamg_solve",
    "aspamg_solve_batch", "aspamg_vcycle", "aspamg_apply_operator", "aspamg_apply_operator_noalloc",
    "aspamg_level_info",
    "aspamg_level_matrix", "aspamg_level_split", "aspamg_level_test_space", "aspamg_element_gradient", "aspamg_assembler_create",
    "aspamg_assemble", "aspamg_assembler_destroy", "aspamg_time_kernel", "aspamg_time_operator", "aspamg_destroy",
    "aspamg_last_error",
]


class Params(C.Structure):
    _fields_ = [
        ("k_g", C.c_int32), ("rho_g", C.c_int32), ("eps_g", C.c_double), ("n_tv", C.c_int32),
        ("n_rq", C.c_int32), ("theta", C.c_int32), ("n_max", C.c_int32), ("kappa_p", C.c_double),
        ("rho_blocks", C.c_int32), ("omega_bar", C.c_double), ("outer_fsai", C.c_int32), ("d_p", C.c_int32),
        ("eps_p", C.c_double), ("lanczos_steps", C.c_int32), ("omega_safety", C.c_double),
        ("coarse_max_dof", C.c_int32), ("max_levels", C.c_int32), ("stall_ratio", C.c_double),
        ("nu1", C.c_int32), ("nu2", C.c_int32), ("cycle_precision", C.c_int32), ("rtol", C.c_double),
        ("max_it", C.c_int32), ("quant_bits", C.c_int32), ("dense_max_dof", C.c_int32),
        ("check_every", C.c_int32), ("use_graph", C.c_int32), ("layout", C.c_int32), ("dense_tail_dof", C.c_int32),
        ("block_size", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iterations", C.c_int32), ("levels", C.c_int32), ("cycle_precision", C.c_int32),
        ("relres_recursive", C.c_double), ("relres_true", C.c_double), ("relres_floor", C.c_double),
        ("t_setup_s", C.c_double),
        ("t_solve_s", C.c_double), ("c_gd", C.c_double), ("c_op", C.c_double), ("c_fs", C.c_double),
        ("bytes_vcycle", C.c_double), ("bytes_iter", C.c_double), ("spmm_tile", C.c_int32),
        ("tail_level", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("n_coarse", C.c_int32), ("nnzb_A", C.c_int64), ("nnzb_G", C.c_int64),
        ("nnzb_P", C.c_int64), ("has_smoother", C.c_int32), ("fsai_rounds", C.c_int32),
        ("lambda1", C.c_double), ("omega_q", C.c_double), ("omega_s", C.c_double),
        ("sell_slots_A", C.c_int64), ("sell_slots_G", C.c_int64), ("sell_slots_GT", C.c_int64),
        ("sell_lanes64", C.c_int32 * 5), ("sell_lanes32", C.c_int32 * 5),
        ("sell_index16", C.c_int32), ("sell_stacked", C.c_int32), ("nnzb_M", C.c_int64),
        ("sell_unit64", C.c_int32 * 5), ("sell_unit32", C.c_int32 * 5),
        ("sell_stacked32", C.c_int32), ("sell_stacked_unit64", C.c_int32), ("sell_stacked_unit32", C.c_int32),
    ]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, C.Array) else v
        return out


class AspamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libaspamg.so (built by paper_1902_01715_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1902_01715_amd/build.py (hipcc, gfx950) first")
        # the library and PyTorch must share one HIP runtime (libamdhip64.so.7):
        # load PyTorch's first so that the library binds to it, not to a second copy
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.aspamg_default_params.argtypes = [C.POINTER(Params)]
        L.aspamg_setup.argtypes = [C.POINTER(Params), C.c_int32, C.c_int64, P, P, P, C.c_int32, P, P,
                                   C.POINTER(C.c_void_p)]
        L.aspamg_set_cycle_precision.argtypes = [P, C.c_int32]
        L.aspamg_solve.argtypes = [P, P, P, C.POINTER(Stats)]
        L.aspamg_solve_batch.argtypes = [P, C.c_int32, P, C.c_int64, P, C.c_int64, P]
        L.aspamg_vcycle.argtypes = [P, P, P]
        L.aspamg_apply_operator.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.aspamg_apply_operator_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.aspamg_level_info.argtypes = [P, C.c_int32, C.POINTER(LevelInfo)]
        L.aspamg_level_matrix.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.aspamg_level_split.argtypes = [P, C.c_int32, P, P, P]
        L.aspamg_level_test_space.argtypes = [P, C.c_int32, P]
        L.aspamg_element_gradient.argtypes = [C.c_int64, P, P, C.c_int64, P, P, P, P, P]
        L.aspamg_assembler_create.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P, C.c_int64, P,
                                              C.POINTER(C.c_void_p)]
        L.aspamg_assemble.argtypes = [P, P, P]
        L.aspamg_assembler_destroy.argtypes = [P]
        L.aspamg_time_kernel.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.aspamg_time_operator.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double)]
        L.aspamg_destroy.argtypes = [P]
        L.aspamg_last_error.restype = C.c_char_p
        for nm in EXPORTED:
            if nm != "aspamg_last_error":
                getattr(L, nm).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, allow_warning=False):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise AspamgError(rc, lib().aspamg_last_error().decode())
    return rc


def default_params(**kw) -> Params:
    p = Params()
    lib().aspamg_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(x):
    """Raw pointer of a numpy array or torch tensor (host or device)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(C.c_void_p)
    return C.c_void_p(x.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Solver:
    """aSP-AMG preconditioned CG for an SPD matrix in b x b block CSR
    (params.block_size: 3, nodal blocks of elasticity; 1, scalar CSR and the
    paper's point-wise rules).

    row_ptr/col/vals: block CSR of K (numpy host arrays or torch device
    tensors; vals [nnzb, b, b]), V0: near-null space [n_nodes, b, n_tv]
    (rigid-body modes for elasticity)."""

    def __init__(self, row_ptr, col, vals, V0, params: Params | None = None, stream=None):
        import torch
        self.params = params if params is not None else default_params()
        self.n = int(len(row_ptr) - 1)
        self.nnzb = int(row_ptr[-1])
        self.b = int(self.params.block_size)
        def host_or_device(a, dtype, tdtype):
            if isinstance(a, np.ndarray):
                return np.ascontiguousarray(a, dtype=dtype)
            assert a.dtype == tdtype, f"expected {tdtype}, got {a.dtype}"
            return a.contiguous()

        row_ptr = host_or_device(row_ptr, np.int32, torch.int32)
        col = host_or_device(col, np.int32, torch.int32)
        vals = host_or_device(vals, np.float64, torch.float64)
        V0 = host_or_device(V0, np.float64, torch.float64)
        n_tv = int(V0.shape[-1])
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().aspamg_setup(C.byref(self.params), self.n, self.nnzb, _ptr(row_ptr), _ptr(col), _ptr(vals),
                                  n_tv, _ptr(V0), _stream_ptr(self._stream), C.byref(h)))
        self.h = h
        self.n_tv = n_tv
        self.precision = int(self.params.cycle_precision)
        self.last_stats = None

    def close(self):
        if getattr(self, "h", None):
            lib().aspamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, bits: int):
        _check(lib().aspamg_set_cycle_precision(self.h, bits))
        self.precision = bits

    def solve(self, f, u=None, check=True):
        """u = K^{-1} f by PCG; f, u float64 CUDA tensors of b n entries."""
        import torch
        assert f.is_cuda and f.dtype == torch.float64 and f.numel() == self.b * self.n
        f = f.contiguous()
        if u is None:
            u = torch.empty_like(f)
        self._stream.synchronize()
        st = Stats()
        rc = lib().aspamg_solve(self.h, _ptr(f), _ptr(u), C.byref(st))
        self.last_stats = st.as_dict()
        if check:
            _check(rc, allow_warning=True)
        return u

    def solve_batch(self, F, U=None):
        """Columns of F [3n, k] solved together; float64 CUDA tensors (block size 3)."""
        import torch
        assert F.is_cuda and F.dtype == torch.float64 and F.shape[0] == self.b * self.n
        F = F.contiguous()
        k = F.shape[1]
        if U is None:
            U = torch.empty_like(F)
        stats = (Stats * k)()
        self._stream.synchronize()
        rc = lib().aspamg_solve_batch(self.h, k, _ptr(F), F.stride(0), _ptr(U), U.stride(0), stats)
        self.last_stats = [s.as_dict() for s in stats]
        _check(rc, allow_warning=True)
        return U

    def vcycle(self, y, z=None):
        import torch
        if z is None:
            z = torch.empty_like(y)
        self._stream.synchronize()
        _check(lib().aspamg_vcycle(self.h, _ptr(y.contiguous()), _ptr(z)))
        return z

    def apply(self, level, which, x, precision=64, out_rows=None):
        """Apply A (0), G (1), G^T (2), P (3), R (4) or the merged G^T G (5) of a level to x."""
        import torch
        info = self.level_info(level)
        if out_rows is None:
            out_rows = self.b * (info["n_coarse"] if which == 4 else info["n"])
        y = torch.empty(out_rows, dtype=torch.float64, device=x.device)
        self._stream.synchronize()
        _check(lib().aspamg_apply_operator(self.h, level, which, precision, _ptr(x.contiguous()), _ptr(y)))
        return y

    def apply_noalloc(self, level, which, x, y, precision=64):
        """The same product as apply() into a caller-provided y, through the
        entry point that allocates no device memory."""
        self._stream.synchronize()
        _check(lib().aspamg_apply_operator_noalloc(self.h, level, which, precision, _ptr(x.contiguous()), _ptr(y)))
        return y

    def time_kernel(self, which, reps=20):
        """(average ms per launch, algorithmic bytes per launch) of a solve-path kernel."""
        ms, by = C.c_double(), C.c_double()
        self._stream.synchronize()
        _check(lib().aspamg_time_kernel(self.h, which, reps, C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def time_operator(self, level, op, precision, reps=20):
        """(average ms per launch, algorithmic bytes per launch) of one V-cycle
        product of a level (op codes of aspamg_time_operator)."""
        ms, by = C.c_double(), C.c_double()
        self._stream.synchronize()
        _check(lib().aspamg_time_operator(self.h, level, op, precision, reps, C.byref(ms), C.byref(by)))
        return ms.value, by.value

    @property
    def nlev(self):
        n = 0
        while True:
            li = LevelInfo()
            if lib().aspamg_level_info(self.h, n, C.byref(li)) != 0:
                return n
            n += 1

    def level_info(self, level):
        li = LevelInfo()
        _check(lib().aspamg_level_info(self.h, level, C.byref(li)))
        return li.as_dict()

    def level_matrix(self, level, which):
        """(row_ptr int64, col int32, vals [nnzb,b,b]) of A (0), G (1) or P (3)."""
        li = self.level_info(level)
        nnz = {0: li["nnzb_A"], 1: li["nnzb_G"], 3: li["nnzb_P"]}[which]
        rp = np.zeros(li["n"] + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros((max(nnz, 1), self.b, self.b))
        _check(lib().aspamg_level_matrix(self.h, level, which, _ptr(rp), _ptr(ci), _ptr(v)))
        return rp, ci[:nnz], v[:nnz]

    def level_split(self, level):
        li = self.level_info(level)
        n = li["n"]
        cf = np.zeros(n, dtype=np.int8)
        cnt = np.zeros(self.b * n, dtype=np.int32)
        cols = np.zeros((self.b * n, self.params.n_max), dtype=np.int32)
        _check(lib().aspamg_level_split(self.h, level, _ptr(cf), _ptr(cnt), _ptr(cols)))
        return cf, cnt, cols

    def level_test_space(self, level):
        """The level's orthonormalised test space, [n, b, n_tv]."""
        n = self.level_info(level)["n"]
        V = np.zeros((n, self.b, self.n_tv))
        _check(lib().aspamg_level_test_space(self.h, level, _ptr(V)))
        return V


def element_gradient(conn, Ke0, lam, u, scale=None, stream=None):
    """grad_e = -scale_e lam_e^T K_e^0 u_e on the GPU (conn int32 [n_el,8], Ke0 [24,24] or [n_el,24,24])."""
    import torch
    n_el = conn.shape[0]
    grad = torch.empty(n_el, dtype=torch.float64, device=lam.device)
    ke_stride = 0 if Ke0.dim() == 2 else 576
    _check(lib().aspamg_element_gradient(n_el, _ptr(conn.contiguous()), _ptr(Ke0.contiguous()), ke_stride,
                                         _ptr(lam.contiguous()), _ptr(u.contiguous()),
                                         _ptr(scale.contiguous()) if scale is not None else None, _ptr(grad),
                                         _stream_ptr(stream)))
    return grad


class Assembler:
    """K(E) = sum_e E_e K_e^0 into a fixed block pattern, on the GPU."""

    def __init__(self, n_nodes, conn, constrained, row_ptr, col, Ke0, stream=None):
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        cons = np.ascontiguousarray(constrained, dtype=np.int8)
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        Ke0 = np.ascontiguousarray(Ke0, dtype=np.float64)
        ke_stride = 0 if Ke0.ndim == 2 else 576
        self.nnzb = int(row_ptr[-1])
        self.stream = stream
        h = C.c_void_p()
        _check(lib().aspamg_assembler_create(n_nodes, conn.shape[0], _ptr(conn), _ptr(cons), _ptr(row_ptr),
                                             _ptr(col), _ptr(Ke0), ke_stride, _stream_ptr(stream), C.byref(h)))
        self.h = h

    def __call__(self, E, vals=None):
        import torch
        if vals is None:
            vals = torch.empty((self.nnzb, 3, 3), dtype=torch.float64, device=E.device)
        _check(lib().aspamg_assemble(self.h, _ptr(E.contiguous()), _ptr(vals)))
        return vals

    def __del__(self):
        if getattr(self, "h", None):
            lib().aspamg_assembler_destroy(self.h)
            self.h = None
