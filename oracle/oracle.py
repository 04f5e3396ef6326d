"""ctypes binding of the plain FP64 CPU oracle (``oracle/mg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over z-planes)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Opts(C.Structure):
    _fields_ = [("n_pre", C.c_int), ("n_post", C.c_int), ("n_cycles", C.c_int), ("n_coarse", C.c_int),
                ("max_cycles", C.c_int), ("bc_order", C.c_int), ("eta", C.c_double), ("hold", C.c_int)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int), ("order_used", C.c_int), ("switched_at", C.c_int), ("status", C.c_int),
                ("r_ref", C.c_double), ("r0", C.c_double), ("r_final", C.c_double),
                ("history", C.c_double * 257)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS"), C.c_int, C.c_int, C.c_int,
                                 C.c_double, C.c_int]
        L.orc_destroy.argtypes = [P]
        L.orc_nlevels.argtypes = [P, C.c_int]
        L.orc_level_dims.argtypes = [P, C.c_int, np.ctypeslib.ndpointer(np.int32)]
        L.orc_level_counts.argtypes = [P, C.c_int, np.ctypeslib.ndpointer(np.int64)]
        L.orc_level_active.argtypes = [P, C.c_int, C.c_int, np.ctypeslib.ndpointer(np.uint8)]
        L.orc_level_diag.argtypes = [P, C.c_int, C.c_int, dp]
        L.orc_smooth.argtypes = [P, C.c_int, C.c_int, dp, dp, P, C.c_int]
        L.orc_residual.argtypes = [P, C.c_int, C.c_int, dp, dp, P, dp]
        L.orc_restrict.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.orc_prolong.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.orc_vcycle.argtypes = [P, C.c_int, dp, dp, P, C.POINTER(Opts)]
        L.orc_residual_norm.restype = C.c_double
        L.orc_residual_norm.argtypes = [P, dp, dp, P]
        L.orc_default_opts.argtypes = [C.POINTER(Opts)]
        L.orc_solve.argtypes = [P, dp, dp, P, C.c_double, C.POINTER(Opts), C.POINTER(Info)]
        L.orc_get_hold.argtypes = [P]
        L.orc_set_hold.argtypes = [P, C.c_int]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "bc_order" and isinstance(v, str):
            v = {"auto": 0, "first": 1, "second": 2}[v]
        setattr(o, k, v)
    return o


def set_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


class Oracle:
    """Hierarchy of the plain oracle.  ``order`` is 1 (first) or 2 (second)."""

    def __init__(self, mask, h, min_coarse_dim: int = 4):
        mask = np.ascontiguousarray(mask, dtype=np.int8)
        nz, ny, nx = mask.shape
        self.shape = mask.shape
        self.h = float(h)
        self._p = lib().orc_create(mask, nx, ny, nz, self.h, int(min_coarse_dim))
        if not self._p:
            raise ValueError("oracle: invalid hierarchy arguments")

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_destroy(self._p)
            self._p = None

    # -- inspection --
    def nlevels(self, order: int = 0) -> int:
        return int(lib().orc_nlevels(self._p, order))

    def dims(self, level: int):
        d = np.zeros(3, np.int32)
        lib().orc_level_dims(self._p, level, d)
        return int(d[2]), int(d[1]), int(d[0])  # (nz, ny, nx)

    def counts(self, level: int) -> np.ndarray:
        out = np.zeros(self.dims(level), np.int64)
        lib().orc_level_counts(self._p, level, out)
        return out

    def active(self, level: int, order: int = 2) -> np.ndarray:
        out = np.zeros(self.dims(level), np.uint8)
        lib().orc_level_active(self._p, level, order, out)
        return out

    def diag(self, level: int, order: int = 2) -> np.ndarray:
        out = np.zeros(self.dims(level), np.float64)
        lib().orc_level_diag(self._p, level, order, out)
        return out

    # -- single operators --
    def smooth(self, level, x, rhs, B=None, passes=1, order=2):
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        B = _f64(B)
        lib().orc_smooth(self._p, level, order, x, _f64(rhs), _ptr(B), int(passes))
        return x

    def residual(self, level, x, rhs, B=None, order=2):
        r = np.zeros(self.dims(level), np.float64)
        B = _f64(B)
        lib().orc_residual(self._p, level, order, _f64(x), _f64(rhs), _ptr(B), r)
        return r

    def restrict(self, level, r, order=2):
        fc = np.zeros(self.dims(level + 1), np.float64)
        lib().orc_restrict(self._p, level, order, _f64(r), fc)
        return fc

    def prolong(self, level, xc, x, order=2):
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        lib().orc_prolong(self._p, level, order, _f64(xc), x)
        return x

    def vcycle(self, phi, rho, B=None, order=2, **opts):
        phi = np.array(phi, dtype=np.float64, copy=True, order="C")
        B = _f64(B)
        o = default_opts(**opts)
        lib().orc_vcycle(self._p, order, phi, _f64(rho), _ptr(B), C.byref(o))
        return phi

    def residual_norm(self, rho, phi, B=None) -> float:
        B = _f64(B)
        return float(lib().orc_residual_norm(self._p, _f64(rho), _f64(phi), _ptr(B)))

    def solve(self, rho, phi=None, B=None, tol=1e-10, **opts):
        """Returns (phi, info dict).  ``phi`` is the initial guess (zeros if None)."""
        rho = _f64(rho)
        phi = np.zeros(self.shape) if phi is None else np.array(phi, dtype=np.float64, copy=True, order="C")
        B = _f64(B)
        o = default_opts(**opts)
        info = Info()
        st = lib().orc_solve(self._p, rho, phi, _ptr(B), float(tol), C.byref(o), C.byref(info))
        n = info.cycles
        return phi, {
            "status": int(st), "cycles": n, "order_used": info.order_used, "switched_at": info.switched_at,
            "r_ref": info.r_ref, "r0": info.r0, "r_final": info.r_final,
            "history": [info.history[i] for i in range(min(n, 256) + 1)],
        }

    @property
    def hold(self) -> int:
        return int(lib().orc_get_hold(self._p))

    @hold.setter
    def hold(self, v: int) -> None:
        lib().orc_set_hold(self._p, int(v))
