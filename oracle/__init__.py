"""CPU ORACLE (test infrastructure only).

Python bindings (ctypes + numpy) for the plain serial FP64 oracle in
oracle.c / unet.c.  Only the tests, the smoke check and the benchmark's CPU
baseline leg use this package; the product path never imports it.  It shares
no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same sources (the mutation tests load
# deliberately broken copies this way, in a subprocess of their own)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
ERR_ARG, ERR_OOM, ERR_ZERO_PIVOT, ERR_NAN, ERR_PATTERN = -1, -2, -4, -5, -6

_lib = None
APPLY_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double))


class Stats(ctypes.Structure):
    _fields_ = [("its", ctypes.c_int64), ("restarts", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
                ("final_relres", ctypes.c_double), ("bad_cell", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "orc_bcsr_from_stencil": ([i32, i32, i32, vp, P(vp)], ctypes.c_int),
        "orc_bcsr_from_dense_pattern": ([i64, vp, vp, vp, P(vp)], ctypes.c_int),
        "orc_bcsr_free": ([vp], None),
        "orc_bcsr_nnzb": ([vp], i64),
        "orc_bcsr_export": ([vp, vp, vp, vp], None),
        "orc_spmv": ([vp, vp, vp], None),
        "orc_ilu0": ([vp, P(vp), P(i64)], ctypes.c_int),
        "orc_ilu_free": ([vp], None),
        "orc_ilu_factors": ([vp], vp),
        "orc_ilu_apply": ([vp, vp, vp], ctypes.c_int),
        "orc_ilu_apply_f32": ([vp, vp, vp], ctypes.c_int),
        "orc_ras_setup": ([vp, i32, i32, i32, i32, i32, i32, i32, P(vp), P(i64)], ctypes.c_int),
        "orc_ras_setup_k": ([vp, i32, i32, i32, i32, i32, i32, i32, i32, P(vp), P(i64)], ctypes.c_int),
        "orc_iluk": ([vp, i32, P(vp), P(i64)], ctypes.c_int),
        "orc_ilut": ([vp, i32, dbl, P(vp), P(i64)], ctypes.c_int),
        "orc_ras_setup_ilut": ([vp, i32, i32, i32, i32, i32, i32, i32, i32, dbl, P(vp), P(i64)], ctypes.c_int),
        "orc_iluk_pattern": ([vp, i32, vp, vp, vp, i64], ctypes.c_int),
        "orc_ras_free": ([vp], None),
        "orc_ras_apply": ([vp, vp, vp], ctypes.c_int),
        "orc_ras_nsub": ([vp], i64),
        "orc_ras_sub_size": ([vp, i64], i64),
        "orc_ras_sub_cells": ([vp, i64, vp], None),
        "orc_ras_owner": ([vp, vp], None),
        "orc_gmres": ([vp, vp, vp, vp, vp, i32, dbl, i64, P(Stats), vp], ctypes.c_int),
        "orc_bicgstab": ([vp, vp, vp, vp, vp, dbl, i64, P(Stats), vp], ctypes.c_int),
        "orc_fgmres": ([vp, vp, vp, vp, vp, dbl, vp, vp, i32, dbl, i64, P(Stats), vp], ctypes.c_int),
        "orc_inv3": ([vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _unet_bind(L)
    _lib = L
    return L


def _unet_bind(L):
    try:
        from . import unet as _u
    except ImportError:  # pragma: no cover
        return
    _u._bind(L)


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, rc, msg=""):
        super().__init__(f"oracle status {rc} {msg}")
        self.rc = rc


class BCSR:
    """Block CSR (3x3 blocks) owned by the oracle library."""

    def __init__(self, handle, n):
        self.h = ctypes.c_void_p(handle)
        self.n = n

    @classmethod
    def from_stencil(cls, nx, ny, nz, blocks):
        blocks = _f64(blocks)
        assert blocks.size == nx * ny * nz * 63
        h = ctypes.c_void_p()
        rc = lib().orc_bcsr_from_stencil(nx, ny, nz, _p(blocks), ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "from_stencil")
        return cls(h.value, nx * ny * nz)

    @classmethod
    def from_csr(cls, rowptr, col, val):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int64)
        val = _f64(val)
        n = len(rowptr) - 1
        h = ctypes.c_void_p()
        rc = lib().orc_bcsr_from_dense_pattern(n, _p(rowptr), _p(col), _p(val), ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "from_csr")
        return cls(h.value, n)

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.orc_bcsr_free(self.h)
            self.h = None

    @property
    def nnzb(self):
        return lib().orc_bcsr_nnzb(self.h)

    def export(self):
        nnzb = self.nnzb
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(nnzb, np.int64)
        val = np.empty((nnzb, 3, 3), np.float64)
        lib().orc_bcsr_export(self.h, _p(rp), _p(col), _p(val))
        return rp, col, val

    def spmv(self, x):
        x = _f64(x)
        y = np.empty(3 * self.n, np.float64)
        lib().orc_spmv(self.h, _p(x), _p(y))
        return y


def bcsr_to_dense(rp, col, val):
    n = len(rp) - 1
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = val[p]
    return D


def iluk_pattern(A: BCSR, k):
    """(rowptr, col, level) of the level-k fill pattern."""
    nnzb = lib().orc_iluk_pattern(A.h, k, None, None, None, 0)
    if nnzb < 0:
        raise OracleError(nnzb, "iluk_pattern")
    rp = np.empty(A.n + 1, np.int64)
    col = np.empty(nnzb, np.int64)
    lev = np.empty(nnzb, np.int64)
    lib().orc_iluk_pattern(A.h, k, _p(rp), _p(col), _p(lev), nnzb)
    return rp, col, lev


class ILU:
    def __init__(self, A: BCSR, level=0, ilut=None):
        """ILU(level) by levels of fill, or ILUT(p, tol) when ilut = (p, tol)."""
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        if ilut is not None:
            rc = lib().orc_ilut(A.h, int(ilut[0]), float(ilut[1]), ctypes.byref(h), ctypes.byref(bad))
        else:
            rc = lib().orc_iluk(A.h, level, ctypes.byref(h), ctypes.byref(bad))
        if rc != OK:
            e = OracleError(rc, f"ilu0 bad_cell={bad.value}")
            e.bad_cell = bad.value
            raise e
        self.h = ctypes.c_void_p(h.value)
        self.n = A.n

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.orc_ilu_free(self.h)
            self.h = None

    def factors(self):
        """(rowptr, col, val): strict lower blocks = L (unit diagonal implied), rest = U."""
        hf = lib().orc_ilu_factors(self.h)
        tmp = BCSR.__new__(BCSR)
        tmp.h = None
        tmp.n = self.n
        nnzb = lib().orc_bcsr_nnzb(hf)
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(nnzb, np.int64)
        val = np.empty((nnzb, 3, 3), np.float64)
        lib().orc_bcsr_export(hf, _p(rp), _p(col), _p(val))
        return rp, col, val

    def apply(self, r, fp32=False):
        r = _f64(r)
        z = np.empty_like(r)
        f = lib().orc_ilu_apply_f32 if fp32 else lib().orc_ilu_apply
        rc = f(self.h, _p(r), _p(z))
        if rc != OK:
            raise OracleError(rc)
        return z

    def fnptr(self, fp32=False):
        name = "orc_ilu_apply_f32" if fp32 else "orc_ilu_apply"
        return ctypes.cast(getattr(lib(), name), ctypes.c_void_p).value, self.h.value


class RAS:
    def __init__(self, A: BCSR, dims, parts, overlap=1, level=0, ilut=None):
        """Local solvers ILU(level), or ILUT(p, tol) when ilut = (p, tol)."""
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        nx, ny, nz = dims
        px, py, pz = parts
        if ilut is not None:
            rc = lib().orc_ras_setup_ilut(A.h, nx, ny, nz, px, py, pz, overlap, int(ilut[0]), float(ilut[1]),
                                          ctypes.byref(h), ctypes.byref(bad))
        else:
            rc = lib().orc_ras_setup_k(A.h, nx, ny, nz, px, py, pz, overlap, level, ctypes.byref(h),
                                       ctypes.byref(bad))
        if rc != OK:
            e = OracleError(rc, f"ras_setup bad_cell={bad.value}")
            e.bad_cell = bad.value
            raise e
        self.h = ctypes.c_void_p(h.value)
        self.n = A.n

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.orc_ras_free(self.h)
            self.h = None

    @property
    def nsub(self):
        return lib().orc_ras_nsub(self.h)

    def sub_cells(self, s):
        m = lib().orc_ras_sub_size(self.h, s)
        out = np.empty(m, np.int64)
        lib().orc_ras_sub_cells(self.h, s, _p(out))
        return out

    def owner(self):
        out = np.empty(self.n, np.int64)
        lib().orc_ras_owner(self.h, _p(out))
        return out

    def apply(self, r):
        r = _f64(r)
        z = np.zeros_like(r)
        rc = lib().orc_ras_apply(self.h, _p(r), _p(z))
        if rc != OK:
            raise OracleError(rc)
        return z

    def fnptr(self):
        return ctypes.cast(lib().orc_ras_apply, ctypes.c_void_p).value, self.h.value


def _pc_args(pc):
    """pc: None | ILU | RAS | (ILU, 'fp32') | python callable(r)->z"""
    keep = None
    if pc is None:
        return None, None, keep
    if isinstance(pc, tuple) and pc[1] == "fp32":
        f, c = pc[0].fnptr(fp32=True)
        return f, c, keep
    if hasattr(pc, "fnptr"):
        f, c = pc.fnptr()
        return f, c, keep
    if callable(pc):
        def cb(ctx, inp, out, _pc=pc):
            n = cb.n
            a = np.ctypeslib.as_array(inp, shape=(n,))
            try:
                z = _pc(a.copy())
            except Exception:  # noqa: BLE001
                return ERR_NAN
            o = np.ctypeslib.as_array(out, shape=(n,))
            o[:] = z
            return OK
        keep = APPLY_FN(cb)
        keep_cb = cb
        return ctypes.cast(keep, ctypes.c_void_p).value, None, (keep, keep_cb)
    raise TypeError(pc)


def _set_n(keep, n):
    if keep is not None:
        keep[1].n = n


def gmres(A: BCSR, b, pc=None, x0=None, m=30, tol=1e-8, maxit=10000, hist=False):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    f, c, keep = _pc_args(pc)
    _set_n(keep, len(b))
    st = Stats()
    h = np.full(maxit + 1, np.nan) if hist else None
    rc = lib().orc_gmres(A.h, f, c, _p(b), _p(x), m, tol, maxit, ctypes.byref(st),
                         _p(h) if hist else None)
    out = {"rc": rc, "x": x, "its": st.its, "restarts": st.restarts, "relres": st.final_relres}
    if hist:
        out["hist"] = h[: st.its + 1]
    return out


def fgmres(A: BCSR, b, pc, fallback, theta=0.99, x0=None, m=30, tol=1e-8, maxit=10000, hist=False):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    f, c, keep = _pc_args(pc)
    _set_n(keep, len(b))
    ff, fc, keep2 = _pc_args(fallback)
    _set_n(keep2, len(b))
    st = Stats()
    h = np.full(maxit + 1, np.nan) if hist else None
    rc = lib().orc_fgmres(A.h, f, c, ff, fc, theta, _p(b), _p(x), m, tol, maxit, ctypes.byref(st),
                          _p(h) if hist else None)
    out = {"rc": rc, "x": x, "its": st.its, "restarts": st.restarts, "relres": st.final_relres,
           "fallbacks": st.fallbacks}
    if hist:
        out["hist"] = h[: st.its + 1]
    return out


def bicgstab(A: BCSR, b, pc=None, x0=None, tol=1e-8, maxit=10000, hist=False):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    f, c, keep = _pc_args(pc)
    _set_n(keep, len(b))
    st = Stats()
    h = np.full(maxit + 1, np.nan) if hist else None
    rc = lib().orc_bicgstab(A.h, f, c, _p(b), _p(x), tol, maxit, ctypes.byref(st),
                            _p(h) if hist else None)
    out = {"rc": rc, "x": x, "its": st.its, "relres": st.final_relres}
    if hist:
        out["hist"] = h[: st.its + 1]
    return out


def inv3(a):
    a = _f64(a).reshape(3, 3)
    out = np.empty((3, 3))
    rc = lib().orc_inv3(_p(a), _p(out))
    return rc, out
