"""Seeded synthetic inputs (permeability fields, 3x3-block 7-point Jacobians,
random vectors).  Inputs only: nothing here multiplies by, factors or solves
with the assembled matrix.  Both the CPU oracle tests and the GPU path read
what this module writes.

The workloads stand in for the paper's SPE1/SPE10-derived reservoir models
(Experiments section), which are not available here: same block structure
(cell-centred structured grid, 7-point stencil, 3 unknowns per cell),
heterogeneous log-normal or channelised permeability.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None

LNK_IID, LNK_LAYERED, LNK_CHANNELS = 0, 1, 2


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lnk_kind", ctypes.c_int32),
        ("sigma", ctypes.c_double), ("sigma_layer", ctypes.c_double),
        ("m_shift", ctypes.c_double),
        ("nsrc", ctypes.c_int32),
        ("src_add", ctypes.c_double), ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"input generator library missing: {_LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.gen_lnk.argtypes = [P(_Cfg), ctypes.c_void_p]
        lib.gen_lnk.restype = ctypes.c_int
        lib.gen_blocks.argtypes = [P(_Cfg), ctypes.c_void_p, ctypes.c_void_p]
        lib.gen_blocks.restype = ctypes.c_int
        lib.gen_uniform_vec.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        lib.gen_uniform_vec.restype = None
        lib.gen_normal_vec.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.gen_normal_vec.restype = None
        lib.gen_poisson.argtypes = [P(_Cfg), ctypes.c_void_p, ctypes.c_void_p]
        lib.gen_poisson.restype = ctypes.c_int
        lib.gen_source_cells.argtypes = [P(_Cfg), ctypes.c_void_p]
        lib.gen_source_cells.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclasses.dataclass
class GenConfig:
    nx: int
    ny: int
    nz: int
    lnk_kind: int = LNK_IID
    sigma: float = 1.0
    sigma_layer: float = 0.0
    m_shift: float = 2.0
    nsrc: int = 0
    src_add: float = 1.0e3
    dt: float = 1.0
    seed: int = 0

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def _c(self) -> _Cfg:
        return _Cfg(self.nx, self.ny, self.nz, self.lnk_kind, self.sigma, self.sigma_layer,
                    self.m_shift, self.nsrc, self.src_add, self.dt, self.seed & (2**64 - 1))

    def replace(self, **kw) -> "GenConfig":
        return dataclasses.replace(self, **kw)


# The five workloads (stand-ins for the paper's reservoir models).
# C1: 20x20x10, ln k ~ N(0,1) iid, GMRES(30)+BILU0.  The literal coupling
#     matrices M ~ U(0.1,1) (shift 0) are the default; the shifted reading
#     (m_shift=2) is run beside it.
# C2: 128x128x64, layered ln k (layer mean ~ N(0,1.5), cell noise ~ N(0,2)),
#     four source cells; BiCGSTAB+BILU0 and GMRES(30)+RAS(64).
# C3: 256x256x128, ln k ~ N(0,3); FP32-factor form vs FP64.
# C4: 64x64x32, ln k ~ N(0,2); learned preconditioner (train / held-out seeds).
# C5: 512x512x128 channelised; eight sources; all three forms.
def preset(name: str, seed: int = 0, m_shift: float | None = None) -> GenConfig:
    name = name.upper()
    if name == "C1":
        c = GenConfig(20, 20, 10, LNK_IID, 1.0, 0.0, 0.0, 0, 1e3, 1.0, seed)   # literal M by default
    elif name == "C2":
        c = GenConfig(128, 128, 64, LNK_LAYERED, 2.0, 1.5, 2.0, 4, 1e3, 1.0, seed)
    elif name == "C3":
        c = GenConfig(256, 256, 128, LNK_IID, 3.0, 0.0, 2.0, 0, 1e3, 1.0, seed)
    elif name == "C4":
        c = GenConfig(64, 64, 32, LNK_IID, 2.0, 0.0, 2.0, 0, 1e3, 1.0, seed)
    elif name == "P1":
        # scalar Poisson (Poisson Equation example): 7-point Laplacian, b = A x_true
        c = GenConfig(512, 512, 512, LNK_IID, 0.0, 0.0, 0.0, 0, 1e3, 1.0, seed)
    elif name == "C5":
        c = GenConfig(512, 512, 128, LNK_CHANNELS, 0.5, 0.0, 2.0, 8, 1e3, 1.0, seed)
    else:
        raise ValueError(name)
    if m_shift is not None:
        c.m_shift = m_shift
    return c


def lnk(cfg: GenConfig) -> np.ndarray:
    lib = _load()
    out = np.empty(cfg.ncell, dtype=np.float64)
    rc = lib.gen_lnk(ctypes.byref(cfg._c()), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"gen_lnk failed ({rc})")
    return out


def blocks(cfg: GenConfig, lnk_field: np.ndarray | None = None) -> np.ndarray:
    """Jacobian blocks, shape (ncell, 7, 3, 3), slots (-z,-y,-x,D,+x,+y,+z)."""
    lib = _load()
    if lnk_field is None:
        lnk_field = lnk(cfg)
    lnk_field = np.ascontiguousarray(lnk_field, dtype=np.float64)
    out = np.empty((cfg.ncell, 7, 3, 3), dtype=np.float64)
    rc = lib.gen_blocks(ctypes.byref(cfg._c()), lnk_field.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"gen_blocks failed ({rc})")
    return out


def poisson(cfg: GenConfig, lnk_field: np.ndarray | None = None) -> np.ndarray:
    """Scalar 7-point coefficients, shape (ncell, 7), slots (-z,-y,-x,D,+x,+y,+z):
    -div(k grad u) with harmonic face transmissibilities and u = 0 outside the
    grid; lnk_field None gives the 7-point Laplacian (k = 1)."""
    lib = _load()
    out = np.empty((cfg.ncell, 7), dtype=np.float64)
    ptr = None if lnk_field is None else np.ascontiguousarray(lnk_field, dtype=np.float64).ctypes.data
    rc = lib.gen_poisson(ctypes.byref(cfg._c()), ptr, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"gen_poisson failed ({rc})")
    return out


def x_true_scalar(cfg: GenConfig) -> np.ndarray:
    """Manufactured solution of a scalar system, U(-1,1) per cell (stream 4)."""
    return uniform(cfg.seed, 4, cfg.ncell, -1.0, 1.0)


def uniform(seed: int, stream: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.float64)
    lib.gen_uniform_vec(seed & (2**64 - 1), stream, n, lo, hi, out.ctypes.data)
    return out


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.float64)
    lib.gen_normal_vec(seed & (2**64 - 1), stream, n, out.ctypes.data)
    return out


def x_true(cfg: GenConfig) -> np.ndarray:
    """Manufactured solution, U(-1,1) per unknown (stream 4)."""
    return uniform(cfg.seed, 4, 3 * cfg.ncell, -1.0, 1.0)


def test_vector(seed: int, n: int, index: int = 0) -> np.ndarray:
    """Random U(-1,1) vector of length n (stream 6, shifted per index)."""
    return uniform(seed * 1000003 + index, 6, n, -1.0, 1.0)


def accumulation(cfg: GenConfig) -> np.ndarray:
    """Accumulation term a[c,p] = U(1,10)/dt (+src_add at sources); A.1 = a."""
    a = uniform(cfg.seed, 3, 3 * cfg.ncell, 1.0, 10.0) / cfg.dt
    srcs = source_cells(cfg)
    a = a.reshape(cfg.ncell, 3)
    for c in srcs:
        a[c, :] += cfg.src_add
    return a.reshape(-1)


def source_cells(cfg: GenConfig) -> list[int]:
    lib = _load()
    buf = np.zeros(8, dtype=np.int64)
    n = lib.gen_source_cells(ctypes.byref(cfg._c()), buf.ctypes.data)
    if n < 0:
        raise ValueError("bad config")
    return [int(v) for v in buf[:n]]
