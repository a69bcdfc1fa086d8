"""ctypes binding of libamg.so (include/amg.h): argument marshalling only.

Every function of the C ABI is exposed under its own name; ``Hierarchy`` is a
thin owner of an ``amg_hierarchy*`` that takes torch device tensors (or raw
device pointers) and forwards them.  There is no fallback: if the HIP library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg.so")

AMG_OK = 0
AMG_ERR_INVALID_ARGUMENT = 1
AMG_ERR_INVALID_MATRIX = 2
AMG_ERR_OUT_OF_MEMORY = 3
AMG_ERR_DEVICE = 4
AMG_ERR_NOT_CONVERGED = 5
AMG_ERR_BREAKDOWN = 6
AMG_ERR_UNSUPPORTED = 7
AMG_PREC_FP64 = 0
AMG_PREC_FP32_INNER = 1
AMG_SMOOTHER_L1 = 0
AMG_SMOOTHER_JACOBI = 1


class amg_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class amg_options(ctypes.Structure):
    _fields_ = [("coarsest_size", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("stall_ratio", ctypes.c_double),
                ("max_aggregate", ctypes.c_int32), ("seed", ctypes.c_uint64), ("kcycle_inner", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("max_coarsest", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("mem_budget", ctypes.c_size_t), ("stream", ctypes.c_void_p),
                ("max_rhs", ctypes.c_int32), ("smoother", ctypes.c_int32), ("jacobi_weight", ctypes.c_double),
                ("autotune", ctypes.c_int32), ("kcycle_threshold", ctypes.c_double), ("skip_ratio", ctypes.c_double),
                ("post_fused", ctypes.c_int32), ("batch_cols", ctypes.c_int32)]


class amg_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]


class amg_group_job(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("column", ctypes.c_int32), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1302_2547_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_sig = {
    "amg_default_options": (None, [ctypes.POINTER(amg_options)]),
    "amg_setup": (ctypes.c_int, [ctypes.POINTER(amg_csr), ctypes.POINTER(amg_options), ctypes.POINTER(_P)]),
    "amg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(amg_solve_info)]),
    "amg_solve_batch": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_double,
                                       ctypes.POINTER(amg_solve_info)]),
    "amg_free": (None, [_P]),
    "amg_grid_laplacian_nnz": (ctypes.c_int64, [ctypes.c_int32, _I32P]),
    "amg_grid_laplacian": (ctypes.c_int, [ctypes.c_int32, _I32P, ctypes.c_double, ctypes.c_uint64, _P, _P, _P, _P]),
    "amg_grid_laplacian_noalloc": (ctypes.c_int, [ctypes.c_int32, _I32P, ctypes.c_double, ctypes.c_uint64, _P, _P,
                                                   _P, _P]),
    "amg_uniform_rhs": (ctypes.c_int, [ctypes.c_int64, ctypes.c_uint64, _P, _P]),
    "amg_release_cached_memory": (None, []),
    "amg_num_levels": (ctypes.c_int, [_P, _I32P]),
    "amg_memory_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "amg_level_sizes": (ctypes.c_int, [_P, ctypes.c_int32, _I32P, _I32P, _I32P]),
    "amg_level_slots": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "amg_export_level": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "amg_spmv": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "amg_kcycle": (ctypes.c_int, [_P, _P, _P]),
    "amg_kcycle_batch": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int32]),
    "amg_solve_group": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(amg_group_job), ctypes.c_double, _P, _I32P,
                                       ctypes.POINTER(amg_solve_info)]),
    "amg_kcycle_group": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(amg_group_job), _P, _I32P]),
    "amg_time_smoother": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    "amg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def device_grid_laplacian(dims, jitter: float = 0.0, seed: int = 0, stream: int | None = None):
    """The grid Laplacian of ``inputs.grid_laplacian(dims, jitter, seed)`` built on
    the current device (bit-identical); returns (row_ptr, col, val) tensors."""
    import torch
    d = len(dims)
    arr = (ctypes.c_int32 * 3)(*[int(v) for v in dims], *([1] * (3 - d)))
    nnz = amg_grid_laplacian_nnz(d, arr)
    if nnz < 0:
        raise ValueError(f"invalid grid {dims}")
    n = 1
    for v in dims:
        n *= int(v)
    dev = torch.device("cuda", torch.cuda.current_device())
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(nnz, dtype=torch.int32, device=dev)
    va = torch.empty(nnz, dtype=torch.float64, device=dev)
    st = amg_grid_laplacian(d, arr, float(jitter), seed & (2**64 - 1), rp.data_ptr(), ci.data_ptr(), va.data_ptr(),
                            stream or 0)
    if st != AMG_OK:
        raise AmgError(st, "amg_grid_laplacian")
    return rp, ci, va


def device_rhs(out, seed: int, stream: int | None = None):
    """out[i] = ``inputs.rhs(n, seed)[i]``, written on the device (asynchronous)."""
    st = amg_uniform_rhs(out.numel(), seed & (2**64 - 1), _ptr(out), stream or 0)
    if st != AMG_OK:
        raise AmgError(st, "amg_uniform_rhs")
    return out


class AmgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {amg_status_string(status).decode()} ({status})")


def _ptr(t) -> int:
    """Raw device pointer of a torch tensor (must be on the GPU) or an int."""
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("libamg takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libamg takes contiguous tensors")
    return t.data_ptr()


def default_options(**kw) -> amg_options:
    o = amg_options()
    amg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


@dataclass
class LevelExport:
    n: int
    nnz: int
    passes: int
    agg: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def _group_jobs(jobs):
    arr = (amg_group_job * max(1, len(jobs)))()
    for k, (h, column, b, x) in enumerate(jobs):
        if b.numel() != h.n or x.numel() != h.n:
            raise ValueError("b and x must have the hierarchy's n entries")
        arr[k] = amg_group_job(h._h.value, column, _ptr(b), _ptr(x))
    return arr


def solve_group(jobs, tol: float = 1e-8, stream: int | None = None, raise_on_error: bool = True):
    """One launch for many solves: jobs is a list of (Hierarchy, column, b, x) with
    float64 device vectors; returns (status, per-job statuses, per-job infos)."""
    arr = _group_jobs(jobs)
    st_out = (ctypes.c_int32 * max(1, len(jobs)))()
    infos = (amg_solve_info * max(1, len(jobs)))()
    st = amg_solve_group(len(jobs), arr, tol, stream or 0, st_out, infos)
    if raise_on_error and st != AMG_OK:
        raise AmgError(st, "amg_solve_group")
    return st, list(st_out)[:len(jobs)], list(infos)[:len(jobs)]


def kcycle_group(jobs, stream: int | None = None):
    """x = B b for every (Hierarchy, column, b, x) job, in one launch."""
    arr = _group_jobs(jobs)
    st_out = (ctypes.c_int32 * max(1, len(jobs)))()
    st = amg_kcycle_group(len(jobs), arr, stream or 0, st_out)
    if st != AMG_OK:
        raise AmgError(st, "amg_kcycle_group")
    return list(st_out)[:len(jobs)]


class Hierarchy:
    """Owns one amg_hierarchy*; tensors are int32/float64 CUDA tensors."""

    def __init__(self, row_ptr, col, val, n: int | None = None, **options):
        import torch
        for t, dt in ((row_ptr, torch.int32), (col, torch.int32), (val, torch.float64)):
            if t.dtype != dt:
                raise TypeError(f"expected {dt}, got {t.dtype}")
        n = row_ptr.numel() - 1 if n is None else n
        self._csr = amg_csr(n, col.numel(), _ptr(row_ptr), _ptr(col), _ptr(val))
        self.options = default_options(**options)
        self._h = _P()
        st = amg_setup(ctypes.byref(self._csr), ctypes.byref(self.options), ctypes.byref(self._h))
        if st != AMG_OK:
            raise AmgError(st, "amg_setup")
        self.n = n

    @property
    def memory_bytes(self) -> int:
        v = ctypes.c_size_t()
        self._check(amg_memory_bytes(self._h, ctypes.byref(v)), "amg_memory_bytes")
        return v.value

    @property
    def num_levels(self) -> int:
        v = ctypes.c_int32()
        self._check(amg_num_levels(self._h, ctypes.byref(v)), "amg_num_levels")
        return v.value

    def level_sizes(self, level: int):
        n, nnz, passes = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(amg_level_sizes(self._h, level, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(passes)),
                    "amg_level_sizes")
        return n.value, nnz.value, passes.value

    def level_slots(self, level: int) -> int:
        """Slots of the level's sliced ELLPACK copy (0: swept in CSR only)."""
        v = ctypes.c_int64()
        self._check(amg_level_slots(self._h, level, ctypes.byref(v)), "amg_level_slots")
        return v.value

    def export_level(self, level: int) -> LevelExport:
        n, nnz, passes = self.level_sizes(level)
        agg = np.empty(n, np.int32)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        va = np.empty(nnz, np.float64)
        self._check(amg_export_level(self._h, level, agg.ctypes.data, rp.ctypes.data, ci.ctypes.data, va.ctypes.data),
                    "amg_export_level")
        return LevelExport(n, nnz, passes, agg, rp, ci, va)

    def solve(self, b, x, tol: float = 1e-8, raise_on_error: bool = True):
        info = amg_solve_info()
        st = amg_solve(self._h, _ptr(b), _ptr(x), tol, ctypes.byref(info))
        if raise_on_error and st not in (AMG_OK,):
            raise AmgError(st, "amg_solve")
        return st, info

    def solve_batch(self, B, X, tol: float = 1e-8, raise_on_error: bool = True):
        """B, X: (nrhs, n) contiguous float64 device tensors (row k = right-hand side k,
        i.e. column-major n x nrhs with leading dimension n)."""
        if B.dim() != 2 or B.shape != X.shape or B.shape[1] != self.n:
            raise ValueError("B and X must both be (nrhs, n)")
        k = B.shape[0]
        infos = (amg_solve_info * k)()
        st = amg_solve_batch(self._h, k, _ptr(B), self.n, _ptr(X), self.n, tol, infos)
        if raise_on_error and st not in (AMG_OK,):
            raise AmgError(st, "amg_solve_batch")
        return st, list(infos)

    def spmv(self, level: int, x, y):
        self._check(amg_spmv(self._h, level, _ptr(x), _ptr(y)), "amg_spmv")

    def kcycle(self, r, z):
        self._check(amg_kcycle(self._h, _ptr(r), _ptr(z)), "amg_kcycle")

    def kcycle_batch(self, R, Z):
        """R, Z: (nrhs, n) contiguous float64 device tensors."""
        if R.dim() != 2 or R.shape != Z.shape or R.shape[1] != self.n:
            raise ValueError("R and Z must both be (nrhs, n)")
        self._check(amg_kcycle_batch(self._h, R.shape[0], _ptr(R), self.n, _ptr(Z), self.n), "amg_kcycle_batch")

    def time_smoother(self, reps: int = 20):
        us, by = ctypes.c_double(), ctypes.c_double()
        self._check(amg_time_smoother(self._h, reps, ctypes.byref(us), ctypes.byref(by)), "amg_time_smoother")
        return us.value, by.value

    def _check(self, st, where):
        if st != AMG_OK:
            raise AmgError(st, where)

    def close(self):
        if self._h:
            amg_free(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
