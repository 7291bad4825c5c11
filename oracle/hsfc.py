"""CPU ORACLE (test infrastructure only): bindings of the Hilbert-curve
partition in hsfc.c."""
from __future__ import annotations

import ctypes

import numpy as np

from . import lib as _oracle_lib

_L = None


def _lib():
    global _L
    if _L is None:
        L = _oracle_lib()
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        for name, args in {"orc_hsfc_key3": [vp, i32, vp], "orc_hsfc_grid_keys": [i32, i32, i32, i32, vp],
                           "orc_hsfc_partition": [i64, vp, i32, vp],
                           "orc_partition_quality": [i32, i32, i32, vp, i32, vp, vp]}.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _L = L
    return _L


def key3(c, levels):
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(1, np.uint64)
    rc = _lib().orc_hsfc_key3(c.ctypes.data, levels, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_hsfc_key3 status {rc}")
    return int(out[0])


def grid_keys(dims, levels):
    nx, ny, nz = dims
    out = np.zeros(nx * ny * nz, np.uint64)
    rc = _lib().orc_hsfc_grid_keys(nx, ny, nz, levels, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_hsfc_grid_keys status {rc}")
    return out


def partition(keys, nparts):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(keys), np.int32)
    rc = _lib().orc_hsfc_partition(len(keys), keys.ctypes.data, nparts, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_hsfc_partition status {rc}")
    return out


def quality(dims, part, nparts):
    """(q, per_part): q = [load imbalance, max b_i/f_i, global surface index,
    average b_i/f_i, max connectivity]; per_part[i] = (|G_i|, f_i, b_i, c_i)."""
    nx, ny, nz = dims
    part = np.ascontiguousarray(part, dtype=np.int32)
    q = np.zeros(5)
    per = np.zeros((nparts, 4), np.int64)
    rc = _lib().orc_partition_quality(nx, ny, nz, part.ctypes.data, nparts, q.ctypes.data, per.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_partition_quality status {rc}")
    return q, per
