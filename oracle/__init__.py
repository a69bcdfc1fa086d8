"""Serial FP64 CPU oracle of unsmoothed-aggregation AMG (ctypes wrapper).

TEST INFRASTRUCTURE: only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never does, and the two share no code.  The arithmetic lives in
``ua_amg_oracle.c`` (plain C, built with gcc); this module only marshals numpy
arrays.  See the header of ``ua_amg_oracle.c`` for what each function follows in
the paper (Sec. 2 eq. (2.4), Sec. 3 Alg. 2 and eq. (3.2), Sec. 4, Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ua_amg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_MATRIX, ERR_NOMEM, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_INTERNAL = 0, 1, 2, 3, 5, 6, 7


_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
# checking build: AddressSanitizer + UndefinedBehaviorSanitizer, any report aborts
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction).  With
    sanitize, a separate instrumented library (load it with the sanitizer runtime
    preloaded and UA_AMG_ORACLE_LIB pointing at it)."""
    lib = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall"] + (SANITIZE_FLAGS if sanitize else [])
                              + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _Options(ctypes.Structure):
    _fields_ = [("coarsest_size", ctypes.c_int), ("max_levels", ctypes.c_int),
                ("stall_ratio", ctypes.c_double), ("max_aggregate", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("kcycle_inner", ctypes.c_int),
                ("smoother", ctypes.c_int), ("jacobi_weight", ctypes.c_double),
                ("kcycle_threshold", ctypes.c_double), ("skip_ratio", ctypes.c_double)]

SMOOTHERS = {"l1": 0, "jacobi": 1}


_lib = None
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(os.environ.get("UA_AMG_ORACLE_LIB") or build())
    c_int, c_double, c_void_p, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64
    lib.orc_splitmix64.argtypes = [c_u64, c_u64]
    lib.orc_splitmix64.restype = c_u64
    lib.orc_fmix32.argtypes = [ctypes.c_uint32]
    lib.orc_fmix32.restype = ctypes.c_uint32
    lib.orc_check_csr.argtypes = [c_int, c_int, _I, _I, _D]
    lib.orc_spmv.argtypes = [c_int, _I, _I, _D, _D, _D]
    lib.orc_spmv.restype = None
    lib.orc_priorities.argtypes = [c_int, _I, _I, c_u64, c_int, _U64]
    lib.orc_priorities.restype = None
    lib.orc_paa.argtypes = [c_int, _I, _I, _U64, c_int, _I, c_void_p]
    lib.orc_number.argtypes = [c_int, _I, _I]
    lib.orc_coarse_operator.argtypes = [c_int, _I, _I, _D, _I, c_int, ctypes.POINTER(ctypes.POINTER(ctypes.c_int)),
                                        ctypes.POINTER(ctypes.POINTER(ctypes.c_int)),
                                        ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
    lib.orc_l1_inverse_diagonal.argtypes = [c_int, _I, _I, _D, _D]
    lib.orc_l1_inverse_diagonal.restype = None
    lib.orc_jacobi_inverse_diagonal.argtypes = [c_int, _I, _I, _D, c_double, _D]
    lib.orc_jacobi_inverse_diagonal.restype = None
    lib.orc_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.orc_default_options.restype = None
    lib.orc_setup.argtypes = [c_int, c_int, _I, _I, _D, ctypes.POINTER(_Options), ctypes.POINTER(c_void_p)]
    lib.orc_free.argtypes = [c_void_p]
    lib.orc_free.restype = None
    lib.orc_num_levels.argtypes = [c_void_p]
    lib.orc_setup_ms.argtypes = [c_void_p]
    lib.orc_setup_ms.restype = c_double
    lib.orc_level_info.argtypes = [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                   ctypes.POINTER(c_int)]
    lib.orc_level_export.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.orc_kcycle_apply.argtypes = [c_void_p, _D, _D]
    lib.orc_solve.argtypes = [c_void_p, _D, _D, c_double, c_int, c_int, ctypes.POINTER(c_int),
                              ctypes.POINTER(c_double), ctypes.POINTER(c_double), c_void_p]
    lib.orc_options_size.restype = c_int
    assert lib.orc_options_size() == ctypes.sizeof(_Options)
    _lib = lib
    return lib


def _csr(rp, ci, va=None):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    if va is None:
        return rp, ci
    return rp, ci, np.ascontiguousarray(va, dtype=np.float64)


# --- primitives --------------------------------------------------------------------------

def splitmix64(seed: int, k: int) -> int:
    return int(_load().orc_splitmix64(seed & (2**64 - 1), k))


def fmix32(h: int) -> int:
    return int(_load().orc_fmix32(h & 0xFFFFFFFF))


def check_csr(rp, ci, va) -> int:
    rp, ci, va = _csr(rp, ci, va)
    return int(_load().orc_check_csr(len(rp) - 1, len(ci), rp, ci, va))


def spmv(rp, ci, va, x):
    rp, ci, va = _csr(rp, ci, va)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(len(rp) - 1)
    _load().orc_spmv(len(rp) - 1, rp, ci, va, x, y)
    return y


def priorities(rp, ci, seed: int, level: int):
    """eq. (3.2) priorities as exact integers 2^32 * 12 * v_i."""
    rp, ci = _csr(rp, ci)
    key = np.empty(len(rp) - 1, dtype=np.uint64)
    _load().orc_priorities(len(rp) - 1, rp, ci, seed & (2**64 - 1), level, key)
    return key


def paa(rp, ci, key, cap: int = 0):
    """Alg. 2 in synchronous passes -> (owner, pass_of, passes)."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    key = np.ascontiguousarray(key, dtype=np.uint64)
    owner = np.empty(n, dtype=np.int32)
    pass_of = np.empty(n, dtype=np.int32)
    passes = _load().orc_paa(n, rp, ci, key, cap, owner, pass_of.ctypes.data)
    if passes < 0:
        raise RuntimeError(f"orc_paa failed: {-passes}")
    return owner, pass_of, int(passes)


def number(owner):
    owner = np.ascontiguousarray(owner, dtype=np.int32)
    agg = np.empty(len(owner), dtype=np.int32)
    nc = _load().orc_number(len(owner), owner, agg)
    return agg, int(nc)


def coarse_operator(rp, ci, va, agg, nc: int):
    """eq. (2.4) -> coarse CSR (rp, ci, va)."""
    rp, ci, va = _csr(rp, ci, va)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    lib = _load()
    p_rp, p_ci = ctypes.POINTER(ctypes.c_int)(), ctypes.POINTER(ctypes.c_int)()
    p_va = ctypes.POINTER(ctypes.c_double)()
    st = lib.orc_coarse_operator(len(rp) - 1, rp, ci, va, agg, nc, ctypes.byref(p_rp), ctypes.byref(p_ci),
                                 ctypes.byref(p_va))
    if st:
        raise RuntimeError(f"orc_coarse_operator failed: {st}")
    crp = np.ctypeslib.as_array(p_rp, shape=(nc + 1,)).copy()
    nnz = int(crp[-1])
    cci = np.ctypeslib.as_array(p_ci, shape=(max(nnz, 1),))[:nnz].copy()
    cva = np.ctypeslib.as_array(p_va, shape=(max(nnz, 1),))[:nnz].copy()
    libc = ctypes.CDLL(None)
    libc.free.argtypes = [ctypes.c_void_p]
    for p in (p_rp, p_ci, p_va):
        libc.free(ctypes.cast(p, ctypes.c_void_p))
    return crp, cci, cva


def l1_inverse_diagonal(rp, ci, va):
    rp, ci, va = _csr(rp, ci, va)
    out = np.empty(len(rp) - 1)
    _load().orc_l1_inverse_diagonal(len(rp) - 1, rp, ci, va, out)
    return out


def jacobi_inverse_diagonal(rp, ci, va, omega):
    rp, ci, va = _csr(rp, ci, va)
    out = np.empty(len(rp) - 1)
    _load().orc_jacobi_inverse_diagonal(len(rp) - 1, rp, ci, va, float(omega), out)
    return out


# --- hierarchy and solve -------------------------------------------------------------------

@dataclass
class Level:
    n: int
    nnz: int
    passes: int
    agg: np.ndarray      # coarse column of each vertex (-1 on the coarsest level)
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    minv: np.ndarray


class Hierarchy:
    """Oracle hierarchy (Alg. 1 setup); owns C memory, freed on close()/del."""

    def __init__(self, rp, ci, va, coarsest_size=64, max_levels=40, stall_ratio=0.9, max_aggregate=0,
                 seed=0x5EED5EED, kcycle_inner=2, smoother="l1", jacobi_weight=2.0 / 3.0, kcycle_threshold=0.0,
                 skip_ratio=0.0):
        lib = _load()
        rp, ci, va = _csr(rp, ci, va)
        opt = _Options()
        lib.orc_default_options(ctypes.byref(opt))
        opt.coarsest_size, opt.max_levels, opt.stall_ratio = coarsest_size, max_levels, stall_ratio
        opt.max_aggregate, opt.seed, opt.kcycle_inner = max_aggregate, seed & (2**64 - 1), kcycle_inner
        opt.smoother, opt.jacobi_weight = SMOOTHERS[smoother], jacobi_weight
        opt.kcycle_threshold = kcycle_threshold
        opt.skip_ratio = skip_ratio
        self._h = ctypes.c_void_p()
        st = lib.orc_setup(len(rp) - 1, len(ci), rp, ci, va, ctypes.byref(opt), ctypes.byref(self._h))
        if st:
            raise RuntimeError(f"orc_setup failed with status {st}")
        self.setup_ms = float(lib.orc_setup_ms(self._h))

    @property
    def num_levels(self) -> int:
        return int(_load().orc_num_levels(self._h))

    def level_info(self, l: int):
        n, nnz, passes = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        st = _load().orc_level_info(self._h, l, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(passes))
        if st:
            raise IndexError(l)
        return n.value, nnz.value, passes.value

    def level(self, l: int) -> Level:
        n, nnz, passes = self.level_info(l)
        agg = np.empty(n, np.int32)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        va = np.empty(nnz, np.float64)
        minv = np.empty(n, np.float64)
        _load().orc_level_export(self._h, l, agg.ctypes.data, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                                 minv.ctypes.data)
        return Level(n, nnz, passes, agg, rp, ci, va, minv)

    def kcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        st = _load().orc_kcycle_apply(self._h, r, z)
        if st:
            raise RuntimeError(f"orc_kcycle_apply failed: {st}")
        return z

    def solve(self, b, x0=None, tol=1e-8, max_iters=200, precond=True, history=False):
        """Outer flexible CG; returns (x, status, iterations, true rel. residual, ms[, history])."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it, rel, ms = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        hist = np.full(max_iters + 1, np.nan) if history else None
        st = _load().orc_solve(self._h, b, x, tol, max_iters, int(bool(precond)), ctypes.byref(it), ctypes.byref(rel),
                               ctypes.byref(ms), hist.ctypes.data if history else None)
        out = (x, int(st), it.value, rel.value, ms.value)
        return out + (hist[: it.value + 1],) if history else out

    def close(self):
        if self._h:
            _load().orc_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
