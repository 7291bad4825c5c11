"""CPU ORACLE (test infrastructure only): bindings of the FP64 U-Net in unet.c."""
from __future__ import annotations

import ctypes

import numpy as np

_L = None


def _bind(L):
    global _L
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "orc_bf16": ([dbl], dbl),
        "orc_conv3d_fwd": ([i32, i32, i32, i32, i32, vp, vp, vp, vp], None),
        "orc_conv3d_bwd": ([i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp], None),
        "orc_unet_nparams": ([i32, i32, i32], i64),
        "orc_unet_forward": ([i32, i32, i32, i32, i32, i32, vp, vp, vp, i32], i32),
        "orc_unet_loss_grad": ([i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, ctypes.POINTER(dbl), i32], i32),
        "orc_unet_prepare": ([i32, i32, i32, vp, vp, vp], dbl),
        "orc_adam": ([i64, vp, vp, vp, vp, i64, dbl], None),
    }
    for name, (a, r) in sig.items():
        if not hasattr(L, name):
            return
        f = getattr(L, name)
        f.argtypes = a
        f.restype = r
    _L = L


def _lib():
    if _L is None:
        from . import lib
        lib()
    return _L


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def bf16(x):
    x = np.asarray(x, dtype=np.float64)
    return np.vectorize(_lib().orc_bf16)(x) if x.ndim else _lib().orc_bf16(float(x))


def bf16_array(x):
    """Vectorised BF16 rounding (ties to even) in numpy, same rule as orc_bf16."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def conv3d(dims, cin, cout, x, w, b=None):
    nx, ny, nz = dims
    x, w = _f(x), _f(w)
    y = np.empty(nx * ny * nz * cout)
    _lib().orc_conv3d_fwd(nx, ny, nz, cin, cout, x.ctypes.data, w.ctypes.data,
                          None if b is None else _f(b).ctypes.data, y.ctypes.data)
    return y


def conv3d_bwd(dims, cin, cout, x, w, dy):
    nx, ny, nz = dims
    x, w, dy = _f(x), _f(w), _f(dy)
    dx = np.empty(nx * ny * nz * cin)
    dw = np.empty(27 * cin * cout)
    db = np.empty(cout)
    _lib().orc_conv3d_bwd(nx, ny, nz, cin, cout, x.ctypes.data, w.ctypes.data, dy.ctypes.data, dx.ctypes.data,
                          dw.ctypes.data, db.ctypes.data)
    return dx, dw, db


def nparams(c0=16, c1=32, c2=64):
    return _lib().orc_unet_nparams(c0, c1, c2)


def forward(params, x0, dims, ch=(16, 32, 64), emulate=False):
    nx, ny, nz = dims
    params, x0 = _f(params), _f(x0)
    y = np.empty(nx * ny * nz * 3)
    rc = _lib().orc_unet_forward(*ch, nx, ny, nz, params.ctypes.data, x0.ctypes.data, y.ctypes.data, int(emulate))
    assert rc == 0, rc
    return y


def loss_grad(params, x0, target, dims, ch=(16, 32, 64), emulate=False):
    nx, ny, nz = dims
    params, x0, target = _f(params), _f(x0), _f(target)
    g = np.empty(len(params))
    loss = ctypes.c_double()
    rc = _lib().orc_unet_loss_grad(*ch, nx, ny, nz, params.ctypes.data, x0.ctypes.data, target.ctypes.data,
                                   g.ctypes.data, ctypes.byref(loss), int(emulate))
    assert rc == 0, rc
    return loss.value, g


def prepare(r, lnk, dims):
    nx, ny, nz = dims
    r, lnk = _f(r), _f(lnk)
    x0 = np.empty(nx * ny * nz * 4)
    s = _lib().orc_unet_prepare(nx, ny, nz, r.ctypes.data, lnk.ctypes.data, x0.ctypes.data)
    return x0, s


def apply(params, r, lnk, dims, ch=(16, 32, 64), emulate=True):
    """z = s * N(r / s, lnk) -- the learned preconditioner's action."""
    x0, s = prepare(r, lnk, dims)
    y = forward(params, x0, dims, ch, emulate)
    return s * y


def adam(p, g, m, v, t, lr):
    p, g, m, v = _f(p).copy(), _f(g), _f(m).copy(), _f(v).copy()
    _lib().orc_adam(len(p), p.ctypes.data, g.ctypes.data, m.ctypes.data, v.ctypes.data, t, lr)
    return p, m, v
