"""CPU ORACLE (test infrastructure only): bindings of mg.c (aggregation
multigrid V-cycle on 7-point scalar systems) and cpr.c (the CPR-type
two-stage preconditioners of the CPR-like Preconditioners subsection)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import BCSR, OracleError
from . import lib as _oracle_lib
from .scalar import CSR

FP, PF, FPF, FFPF = 0, 1, 2, 3
DECOUPLE_NONE, DECOUPLE_QUASI_IMPES, DECOUPLE_ABF = 0, 1, 2

_L = None


def _lib():
    global _L
    if _L is None:
        L = _oracle_lib()
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        sig = {
            "orc_mg_setup": ([vp, i32, i32, i32, i32, i32, i32, P(vp)], ctypes.c_int),
            "orc_mg_free": ([vp], None),
            "orc_mg_apply": ([vp, vp, vp], ctypes.c_int),
            "orc_mg_levels": ([vp], i32),
            "orc_mg_level_dims": ([vp, i32, vp], None),
            "orc_mg_level_matrix": ([vp, i32], vp),
            "orc_mg_gs_sweep": ([vp, vp, vp, i32], ctypes.c_int),
            "orc_cpr_setup": ([vp, i32, i32, i32, i32, i32, vp, vp, i32, i32, i32, P(vp), P(i64)], ctypes.c_int),
            "orc_cpr_free": ([vp], None),
            "orc_cpr_apply": ([vp, vp, vp], ctypes.c_int),
            "orc_cpr_weights": ([vp, vp], None),
            "orc_cpr_pressure_matrix": ([vp], vp),
            "orc_cpr_mg": ([vp], vp),
            "orc_csr_nnz": ([vp], i64),
            "orc_csr_export": ([vp, vp, vp, vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _L = L
    return _L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _export(h, n):
    nnz = _lib().orc_csr_nnz(h)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int64)
    val = np.empty(nnz)
    _lib().orc_csr_export(h, rp.ctypes.data, col.ctypes.data, val.ctypes.data)
    return rp, col, val


def _dense(h, n):
    rp, col, val = _export(h, n)
    D = np.zeros((n, n))
    for i in range(n):
        D[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return D


class _Levels:
    def _levels_of(self, hmg):
        out = []
        for lv in range(_lib().orc_mg_levels(hmg)):
            d = np.zeros(3, np.int32)
            _lib().orc_mg_level_dims(hmg, lv, d.ctypes.data)
            out.append(tuple(int(v) for v in d))
        return out


class MG(_Levels):
    """One V-cycle of the aggregation multigrid for a scalar 7-point CSR matrix."""

    def __init__(self, A: CSR, dims, coarse_max=128, pre=1, post=1):
        h = ctypes.c_void_p()
        rc = _lib().orc_mg_setup(A.h, *dims, coarse_max, pre, post, ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "mg_setup")
        self.h = h
        self.A = A        # the hierarchy keeps a pointer to level 0
        self.n = A.n

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _L is not None:
            _L.orc_mg_free(self.h)
            self.h = None

    def levels(self):
        return self._levels_of(self.h)

    def level_dense(self, lv):
        d = self.levels()[lv]
        return _dense(_lib().orc_mg_level_matrix(self.h, lv), d[0] * d[1] * d[2])

    def level_csr(self, lv):
        d = self.levels()[lv]
        return _export(_lib().orc_mg_level_matrix(self.h, lv), d[0] * d[1] * d[2])

    def gs_sweep(self, b, x, colour):
        b = _f64(b)
        x = _f64(x).copy()
        rc = _lib().orc_mg_gs_sweep(self.h, b.ctypes.data, x.ctypes.data, colour)
        if rc != 0:
            raise OracleError(rc)
        return x

    def apply(self, b):
        b = _f64(b)
        x = np.empty_like(b)
        rc = _lib().orc_mg_apply(self.h, b.ctypes.data, x.ctypes.data)
        if rc != 0:
            raise OracleError(rc)
        return x

    def fnptr(self):
        return ctypes.cast(_lib().orc_mg_apply, ctypes.c_void_p).value, self.h.value


class CPR(_Levels):
    """CPR-type preconditioner of a block matrix; R is an oracle
    preconditioner object of the whole system (ILU, RAS) with fnptr()."""

    def __init__(self, A: BCSR, dims, R, variant=FPF, decouple=DECOUPLE_NONE, coarse_max=128, pre=1, post=1):
        f, c = R.fnptr()
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        rc = _lib().orc_cpr_setup(A.h, *dims, variant, decouple, f, c, coarse_max, pre, post, ctypes.byref(h),
                                  ctypes.byref(bad))
        if rc != 0:
            e = OracleError(rc, f"cpr_setup bad_cell={bad.value}")
            e.bad_cell = bad.value
            raise e
        self.h = h
        self.A = A
        self.R = R        # kept alive: the oracle holds its function and context
        self.n = A.n
        self.dims = tuple(dims)

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _L is not None:
            _L.orc_cpr_free(self.h)
            self.h = None

    def weights(self):
        w = np.empty((self.n, 3))
        _lib().orc_cpr_weights(self.h, w.ctypes.data)
        return w

    def pressure_csr(self):
        return _export(_lib().orc_cpr_pressure_matrix(self.h), self.n)

    def pressure_dense(self):
        return _dense(_lib().orc_cpr_pressure_matrix(self.h), self.n)

    def levels(self):
        return self._levels_of(_lib().orc_cpr_mg(self.h))

    def apply(self, f):
        f = _f64(f)
        x = np.empty_like(f)
        rc = _lib().orc_cpr_apply(self.h, f.ctypes.data, x.ctypes.data)
        if rc != 0:
            raise OracleError(rc)
        return x

    def fnptr(self):
        return ctypes.cast(_lib().orc_cpr_apply, ctypes.c_void_p).value, self.h.value
