"""CPU ORACLE (test infrastructure only): bindings of the scalar routines in
scalar.c (CSR storage, ILU(0), RAS, GMRES and BiCGSTAB on a scalar
operator)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import OracleError, Stats, _pc_args, _set_n
from . import lib as _oracle_lib

_L = None


def _lib():
    global _L
    if _L is None:
        L = _oracle_lib()
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "orc_csr_from_stencil": ([i32, i32, i32, vp, P(vp)], ctypes.c_int),
            "orc_csr_free": ([vp], None),
            "orc_csr_nnz": ([vp], i64),
            "orc_csr_export": ([vp, vp, vp, vp], None),
            "orc_csr_spmv": ([vp, vp, vp], None),
            "orc_csr_from_arrays": ([i64, vp, vp, vp, P(vp)], ctypes.c_int),
            "orc_csr_ilu0": ([vp, P(vp), P(i64)], ctypes.c_int),
            "orc_silu_free": ([vp], None),
            "orc_silu_factors": ([vp], vp),
            "orc_silu_apply": ([vp, vp, vp], ctypes.c_int),
            "orc_sras_setup": ([vp, i32, i32, i32, i32, i32, i32, i32, P(vp), P(i64)], ctypes.c_int),
            "orc_sras_free": ([vp], None),
            "orc_sras_nsub": ([vp], i64),
            "orc_sras_sub_size": ([vp, i64], i64),
            "orc_sras_sub_cells": ([vp, i64, vp], None),
            "orc_sras_apply": ([vp, vp, vp], ctypes.c_int),
            "orc_csr_gmres": ([vp, vp, vp, vp, vp, i32, dbl, i64, P(Stats), vp], ctypes.c_int),
            "orc_csr_bicgstab": ([vp, vp, vp, vp, vp, dbl, i64, P(Stats), vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _L = L
    return _L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class CSR:
    """Scalar CSR matrix owned by the oracle library."""

    def __init__(self, nx, ny, nz, coef):
        coef = _f64(coef)
        assert coef.size == nx * ny * nz * 7
        h = ctypes.c_void_p()
        rc = _lib().orc_csr_from_stencil(nx, ny, nz, coef.ctypes.data, ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "csr_from_stencil")
        self.h = h
        self.n = nx * ny * nz
        self.dims = (nx, ny, nz)

    @classmethod
    def from_arrays(cls, rowptr, col, val, dims):
        """A copy of a CSR matrix given by its arrays, on an nx x ny x nz grid."""
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int64)
        val = _f64(val)
        n = len(rowptr) - 1
        assert n == dims[0] * dims[1] * dims[2]
        h = ctypes.c_void_p()
        rc = _lib().orc_csr_from_arrays(n, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "csr_from_arrays")
        self = cls.__new__(cls)
        self.h = h
        self.n = n
        self.dims = tuple(dims)
        return self

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _L is not None:
            _L.orc_csr_free(self.h)
            self.h = None

    def export(self):
        nnz = _lib().orc_csr_nnz(self.h)
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(nnz, np.int64)
        val = np.empty(nnz)
        _lib().orc_csr_export(self.h, rp.ctypes.data, col.ctypes.data, val.ctypes.data)
        return rp, col, val

    def dense(self):
        rp, col, val = self.export()
        D = np.zeros((self.n, self.n))
        for i in range(self.n):
            D[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
        return D

    def spmv(self, x):
        x = _f64(x)
        y = np.empty(self.n)
        _lib().orc_csr_spmv(self.h, x.ctypes.data, y.ctypes.data)
        return y


class ILU:
    def __init__(self, A: CSR):
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        rc = _lib().orc_csr_ilu0(A.h, ctypes.byref(h), ctypes.byref(bad))
        if rc != 0:
            e = OracleError(rc, f"csr_ilu0 bad_row={bad.value}")
            e.bad_row = bad.value
            raise e
        self.h = h
        self.n = A.n

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _L is not None:
            _L.orc_silu_free(self.h)
            self.h = None

    def factors(self):
        hf = _lib().orc_silu_factors(self.h)
        nnz = _lib().orc_csr_nnz(hf)
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(nnz, np.int64)
        val = np.empty(nnz)
        _lib().orc_csr_export(hf, rp.ctypes.data, col.ctypes.data, val.ctypes.data)
        return rp, col, val

    def apply(self, r):
        r = _f64(r)
        z = np.empty_like(r)
        rc = _lib().orc_silu_apply(self.h, r.ctypes.data, z.ctypes.data)
        if rc != 0:
            raise OracleError(rc)
        return z

    def fnptr(self):
        return ctypes.cast(_lib().orc_silu_apply, ctypes.c_void_p).value, self.h.value


class RAS:
    def __init__(self, A: CSR, dims, parts, overlap=1):
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        rc = _lib().orc_sras_setup(A.h, *dims, *parts, overlap, ctypes.byref(h), ctypes.byref(bad))
        if rc != 0:
            e = OracleError(rc, f"sras_setup bad_row={bad.value}")
            e.bad_row = bad.value
            raise e
        self.h = h
        self.n = A.n

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _L is not None:
            _L.orc_sras_free(self.h)
            self.h = None

    @property
    def nsub(self):
        return _lib().orc_sras_nsub(self.h)

    def sub_cells(self, s):
        m = _lib().orc_sras_sub_size(self.h, s)
        out = np.empty(m, np.int64)
        _lib().orc_sras_sub_cells(self.h, s, out.ctypes.data)
        return out

    def apply(self, r):
        r = _f64(r)
        z = np.zeros_like(r)
        rc = _lib().orc_sras_apply(self.h, r.ctypes.data, z.ctypes.data)
        if rc != 0:
            raise OracleError(rc)
        return z

    def fnptr(self):
        return ctypes.cast(_lib().orc_sras_apply, ctypes.c_void_p).value, self.h.value


def _pc(pc):
    if hasattr(pc, "fnptr"):
        f, c = pc.fnptr()
        return f, c, None
    return _pc_args(pc)


def gmres(A: CSR, b, pc=None, x0=None, m=30, tol=1e-8, maxit=10000, hist=False):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    f, c, keep = _pc(pc)
    _set_n(keep, len(b))
    st = Stats()
    h = np.full(maxit + 1, np.nan) if hist else None
    rc = _lib().orc_csr_gmres(A.h, f, c, b.ctypes.data, x.ctypes.data, m, tol, maxit, ctypes.byref(st),
                              h.ctypes.data if hist else None)
    out = {"rc": rc, "x": x, "its": st.its, "restarts": st.restarts, "relres": st.final_relres}
    if hist:
        out["hist"] = h[: st.its + 1]
    return out


def bicgstab(A: CSR, b, pc=None, x0=None, tol=1e-8, maxit=10000, hist=False):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    f, c, keep = _pc(pc)
    _set_n(keep, len(b))
    st = Stats()
    h = np.full(maxit + 1, np.nan) if hist else None
    rc = _lib().orc_csr_bicgstab(A.h, f, c, b.ctypes.data, x.ctypes.data, tol, maxit, ctypes.byref(st),
                                 h.ctypes.data if hist else None)
    out = {"rc": rc, "x": x, "its": st.its, "relres": st.final_relres}
    if hist:
        out["hist"] = h[: st.its + 1]
    return out
