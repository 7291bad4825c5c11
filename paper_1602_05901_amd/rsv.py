"""Thin Python binding of the rsv C ABI (include/rsv.h).

Argument marshalling only: every step of the solver runs in the HIP library
librsv.so.  PyTorch supplies device memory (tensor.data_ptr()) and the HIP
stream (torch.cuda.current_stream().cuda_stream).  If the library is missing
this module raises on use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsv.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
ERR_ARG, ERR_OOM, ERR_HIP, ERR_ZERO_PIVOT, ERR_NAN, ERR_PATTERN, ERR_TIMEOUT = -1, -2, -3, -4, -5, -6, -7
BOTTOM_UP, TOP_DOWN = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
PC_NONE, PC_BILU0, PC_RAS, PC_LEARNED, PC_CPR = 0, 1, 2, 3, 4
CPR_FP, CPR_PF, CPR_FPF, CPR_FFPF = 0, 1, 2, 3
DECOUPLE_NONE, DECOUPLE_QUASI_IMPES, DECOUPLE_ABF = 0, 1, 2
LOCAL_ILUK, LOCAL_ILUT = 0, 1
FP64, FP32 = 0, 1
GMRES, BICGSTAB, FGMRES = 0, 1, 2
CGS2, DCGS2 = 0, 1

vp, i32, i64, dbl, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64


class PcParams(ctypes.Structure):
    _fields_ = [("type", i32), ("precision", i32), ("ras_px", i32), ("ras_py", i32), ("ras_pz", i32),
                ("ras_overlap", i32), ("iluk_level", i32), ("pipelined", i32), ("net", vp), ("lnk", vp),
                ("theta", dbl), ("learned_mode", i32), ("ras_stack", i32), ("ras_group", i32),
                ("cpr_variant", i32), ("cpr_stage", i32), ("cpr_decouple", i32), ("mg_pre", i32),
                ("mg_post", i32), ("mg_coarse", i32), ("local_solver", i32), ("ilut_p", i32), ("ilut_tol", dbl),
                ("reserved", i32 * 4)]


class SolverParams(ctypes.Structure):
    _fields_ = [("method", i32), ("restart", i32), ("tol", dbl), ("maxit", i64), ("rtol", dbl), ("atol", dbl),
                ("record_history", i32), ("ortho", i32), ("reserved", i32 * 6)]


class Stats(ctypes.Structure):
    _fields_ = [("its", i64), ("restarts", i64), ("fallbacks", i64), ("final_relres", dbl), ("solve_ms", dbl),
                ("bad_cell", i64), ("status", i32), ("reserved", i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class NetArch(ctypes.Structure):
    _fields_ = [("levels", i32), ("c0", i32), ("c1", i32), ("c2", i32), ("reserved", i32 * 4)]


_P = ctypes.POINTER
_SIGS = {
    "rsv_version": ([], i32),
    "rsv_status_str": ([i32], ctypes.c_char_p),
    "rsv_last_error": ([vp], ctypes.c_char_p),
    "rsv_create": ([i32, _P(vp)], i32),
    "rsv_set_stream": ([vp, vp], i32),
    "rsv_destroy": ([vp], None),
    "rsv_grid_create": ([vp, i32, i32, i32, i32, _P(vp)], i32),
    "rsv_grid_destroy": ([vp], None),
    "rsv_grid_ncell": ([vp], i64),
    "rsv_cell_to_row": ([vp, i32, i32, i32, _P(i64)], i32),
    "rsv_row_to_cell": ([vp, i64, _P(i32), _P(i32), _P(i32)], i32),
    "rsv_matrix_assemble": ([vp, vp, i32, _P(vp)], i32),
    "rsv_matrix_update": ([vp, vp, i32], i32),
    "rsv_matrix_assemble_scalar": ([vp, vp, i32, _P(vp)], i32),
    "rsv_matrix_destroy": ([vp], None),
    "rsv_spmv": ([vp, dbl, vp, dbl, vp], i32),
    "rsv_spmv_noalloc": ([vp, dbl, vp, dbl, vp], i32),
    "rsv_axpby": ([vp, i64, dbl, vp, dbl, vp], i32),
    "rsv_hsfc_keys": ([vp, i64, vp, i32, vp], i32),
    "rsv_grid_hsfc_keys": ([vp, i32, vp], i32),
    "rsv_hsfc_partition": ([vp, i64, vp, i32, i32, vp], i32),
    "rsv_partition_quality": ([vp, vp, i32, vp, vp], i32),
    "rsv_matrix_device_bytes": ([vp], i64),
    "rsv_pc_params_default": ([_P(PcParams)], None),
    "rsv_precond_setup": ([vp, _P(PcParams), _P(vp), _P(i64)], i32),
    "rsv_precond_apply": ([vp, vp, vp], i32),
    "rsv_precond_bilu0_factors": ([vp, vp, vp], i32),
    "rsv_precond_apply_bytes": ([vp], i64),
    "rsv_cpr_levels": ([vp, _P(i32), vp, i32], i32),
    "rsv_cpr_pressure_matrix": ([vp, i32, vp], i32),
    "rsv_cpr_weights": ([vp, vp], i32),
    "rsv_cpr_pressure_apply": ([vp, vp, vp], i32),
    "rsv_precond_destroy": ([vp], None),
    "rsv_solver_params_default": ([_P(SolverParams)], None),
    "rsv_solve": ([vp, vp, _P(SolverParams), vp, vp, _P(Stats)], i32),
    "rsv_solve_history": ([vp, vp, i64], i64),
    "rsv_net_create": ([vp, _P(NetArch), u64, _P(vp)], i32),
    "rsv_net_destroy": ([vp], None),
    "rsv_net_num_params": ([vp], i64),
    "rsv_net_get_params": ([vp, vp, i64], i32),
    "rsv_net_set_params": ([vp, vp, i64], i32),
    "rsv_net_save": ([vp, ctypes.c_char_p], i32),
    "rsv_net_load": ([vp, ctypes.c_char_p], i32),
    "rsv_net_forward": ([vp, vp, vp, vp, vp], i32),
    "rsv_net_train_step": ([vp, vp, i32, vp, vp, vp, ctypes.c_float, _P(ctypes.c_float)], i32),
    "rsv_net_loss_grad": ([vp, vp, i32, vp, vp, vp, _P(ctypes.c_float), vp], i32),
    "rsv_conv3d": ([vp, i32, i32, i32, i32, i32, vp, vp, vp, vp], i32),
    "rsv_conv3d_bwd": ([vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp], i32),
    "rsv_profile_enable": ([vp, i32], i32),
    "rsv_profile_read": ([vp, vp, vp], i32),
    "rsv_profile_classes": ([vp, ctypes.c_uint32], i32),
    "rsv_device_info": ([vp, vp, i32], i32),
    "rsv_set_wait_limit": ([vp, ctypes.c_double], i32),
}
K_NAMES = ["spmv", "ilu_fwd", "ilu_bwd", "ras", "ortho", "vec", "factor", "net", "cpr"]

_lib = None


def lib():
    """Load librsv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} -- run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class RsvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().rsv_status_str(status).decode()}: {msg}")
        self.status = status


def _check(ctx, status, allow=(OK,)):
    if status not in allow:
        msg = lib().rsv_last_error(ctx.h if ctx is not None else None).decode(errors="replace")
        raise RsvError(status, msg)
    return status


def _ptr(t):
    """Device (or host) address of a torch tensor / numpy array / int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


class Context:
    def __init__(self, device=0, stream=None):
        h = vp()
        _check(None, lib().rsv_create(device, ctypes.byref(h)))
        self.h = h
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        _check(self, lib().rsv_set_stream(self.h, stream))

    def device_info(self):
        import numpy as np
        v = np.zeros(5, np.int64)
        _check(self, lib().rsv_device_info(self.h, v.ctypes.data, 5))
        return {"num_cu": int(v[0]), "lds_per_workgroup": int(v[1]), "lds_per_cu": int(v[2]),
                "sweep_ring_fwd": int(v[3]), "sweep_ring_bwd": int(v[4])}

    def set_wait_limit(self, seconds):
        _check(self, lib().rsv_set_wait_limit(self.h, seconds))

    def profile(self, on=True, classes=None):
        """classes: names from K_NAMES to record (None: all)."""
        mask = 0xFFFFFFFF if classes is None else sum(1 << K_NAMES.index(k) for k in classes)
        _check(self, lib().rsv_profile_classes(self.h, mask))
        _check(self, lib().rsv_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        import numpy as np
        ms = np.zeros(len(K_NAMES))
        cnt = np.zeros(len(K_NAMES), np.int64)
        _check(self, lib().rsv_profile_read(self.h, ms.ctypes.data, cnt.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(K_NAMES)}

    def close(self):
        if self.h:
            lib().rsv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def axpby(ctx: "Context", alpha, x, beta, y):
    """y = alpha x + beta y on device tensors (the library's vector update)."""
    _check(ctx, lib().rsv_axpby(ctx.h, y.numel(), alpha, _ptr(x), beta, _ptr(y)))
    return y


def hsfc_keys(ctx: "Context", coords, levels, keys):
    """Hilbert keys of points (coords: device [n, 3] float64 in [0,1]; keys: device int64 [n])."""
    _check(ctx, lib().rsv_hsfc_keys(ctx.h, keys.numel(), _ptr(coords), levels, _ptr(keys)))
    return keys


def hsfc_partition(ctx: "Context", keys, levels, nparts, part):
    """Equal-count cut of the curve (keys: device int64 [n]; part: device int32 [n])."""
    _check(ctx, lib().rsv_hsfc_partition(ctx.h, keys.numel(), _ptr(keys), levels, nparts, _ptr(part)))
    return part


class Grid:
    def __init__(self, ctx: Context, nx, ny, nz, ordering=BOTTOM_UP):
        h = vp()
        _check(ctx, lib().rsv_grid_create(ctx.h, nx, ny, nz, ordering, ctypes.byref(h)))
        self.ctx, self.h, self.dims = ctx, h, (nx, ny, nz)

    @property
    def ncell(self):
        return lib().rsv_grid_ncell(self.h)

    def hsfc_keys(self, levels, keys):
        """Hilbert keys of the cells (device int64 [ncell], block-row order)."""
        _check(self.ctx, lib().rsv_grid_hsfc_keys(self.h, levels, _ptr(keys)))
        return keys

    def partition_quality(self, part, nparts):
        """(q[5], per_part [nparts, 4]) of a partition (device int32 [ncell])."""
        import numpy as np
        q = np.zeros(5)
        per = np.zeros((nparts, 4), np.int64)
        _check(self.ctx, lib().rsv_partition_quality(self.h, _ptr(part), nparts, q.ctypes.data, per.ctypes.data))
        return q, per

    def cell_to_row(self, i, j, k):
        r = i64()
        _check(self.ctx, lib().rsv_cell_to_row(self.h, i, j, k, ctypes.byref(r)))
        return r.value

    def row_to_cell(self, row):
        i, j, k = i32(), i32(), i32()
        _check(self.ctx, lib().rsv_row_to_cell(self.h, row, ctypes.byref(i), ctypes.byref(j), ctypes.byref(k)))
        return i.value, j.value, k.value

    def close(self):
        if self.h:
            lib().rsv_grid_destroy(self.h)
            self.h = None


class Matrix:
    def __init__(self, grid: Grid, blocks, where=None, scalar=False):
        """blocks: [ncell,7,3,3] float64 (3x3-block system) or, with scalar=True,
        [ncell,7] float64 coefficients of a scalar system; numpy (host) or torch
        (host or device)."""
        if where is None:
            where = MEM_DEVICE if (hasattr(blocks, "is_cuda") and blocks.is_cuda) else MEM_HOST
        h = vp()
        fn = lib().rsv_matrix_assemble_scalar if scalar else lib().rsv_matrix_assemble
        _check(grid.ctx, fn(grid.h, _ptr(blocks), where, ctypes.byref(h)))
        self.grid, self.ctx, self.h, self.scalar = grid, grid.ctx, h, scalar

    def update(self, blocks, where=None):
        if where is None:
            where = MEM_DEVICE if (hasattr(blocks, "is_cuda") and blocks.is_cuda) else MEM_HOST
        _check(self.ctx, lib().rsv_matrix_update(self.h, _ptr(blocks), where))

    def spmv(self, x, y, alpha=1.0, beta=0.0):
        _check(self.ctx, lib().rsv_spmv(self.h, alpha, _ptr(x), beta, _ptr(y)))
        return y

    def spmv_noalloc(self, x, y, alpha=1.0, beta=0.0):
        """The same product with the library's fixed per-device scratch (no allocation)."""
        _check(self.ctx, lib().rsv_spmv_noalloc(self.h, alpha, _ptr(x), beta, _ptr(y)))
        return y

    @property
    def device_bytes(self):
        return lib().rsv_matrix_device_bytes(self.h)

    def close(self):
        if self.h:
            lib().rsv_matrix_destroy(self.h)
            self.h = None


def pc_params(**kw) -> PcParams:
    p = PcParams()
    lib().rsv_pc_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("net", "lnk"):
            v = _ptr(v) if not isinstance(v, Net) else v.h.value
        setattr(p, k, v)
    return p


def solver_params(**kw) -> SolverParams:
    p = SolverParams()
    lib().rsv_solver_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Precond:
    def __init__(self, A: Matrix, **kw):
        p = pc_params(**kw)
        h = vp()
        bad = i64(-1)
        st = lib().rsv_precond_setup(A.h, ctypes.byref(p), ctypes.byref(h), ctypes.byref(bad))
        if st != OK:
            e = RsvError(st, lib().rsv_last_error(A.ctx.h).decode(errors="replace"))
            e.bad_cell = bad.value
            raise e
        self.A, self.ctx, self.h, self.params = A, A.ctx, h, p
        self._keep = kw

    def apply(self, r, z):
        _check(self.ctx, lib().rsv_precond_apply(self.h, _ptr(r), _ptr(z)))
        return z

    def bilu0_factors(self):
        """(L [ncell, 3, 3, 3] toward -z, -y, -x; Dinv [ncell, 3, 3]) in block-row order
        (FP64 BILU0 only)."""
        import numpy as np
        n = self.A.grid.ncell
        L = np.zeros((n, 3, 3, 3))
        D = np.zeros((n, 3, 3))
        _check(self.ctx, lib().rsv_precond_bilu0_factors(self.h, L.ctypes.data, D.ctypes.data))
        return L, D

    @property
    def apply_bytes(self):
        """Algorithmic bytes of one apply (level-scheduled local solvers), else -1."""
        return lib().rsv_precond_apply_bytes(self.h)

    def cpr_levels(self):
        """Grids (nx, ny, nz) of the CPR pressure multigrid, finest first."""
        import numpy as np
        nl = i32(0)
        dims = np.zeros(3 * 64, np.int32)
        _check(self.ctx, lib().rsv_cpr_levels(self.h, ctypes.byref(nl), dims.ctypes.data, 64))
        return [tuple(int(v) for v in dims[3 * l:3 * l + 3]) for l in range(nl.value)]

    def cpr_pressure_matrix(self, level=0):
        """[n_level, 7] coefficients of the pressure matrix on one level (row order)."""
        import numpy as np
        d = self.cpr_levels()[level]
        out = np.zeros((d[0] * d[1] * d[2], 7))
        _check(self.ctx, lib().rsv_cpr_pressure_matrix(self.h, level, out.ctypes.data))
        return out

    def cpr_weights(self):
        import numpy as np
        out = np.zeros((self.A.grid.ncell, 3))
        _check(self.ctx, lib().rsv_cpr_weights(self.h, out.ctypes.data))
        return out

    def cpr_pressure_apply(self, b, x):
        _check(self.ctx, lib().rsv_cpr_pressure_apply(self.h, _ptr(b), _ptr(x)))
        return x

    def close(self):
        if self.h:
            lib().rsv_precond_destroy(self.h)
            self.h = None


def solve(A: Matrix, M: Precond | None, b, x, allow=(OK, NOT_CONVERGED, BREAKDOWN), **kw):
    """x (device tensor) holds x0 on entry and the result on exit; returns stats dict."""
    p = solver_params(**kw)
    st = Stats()
    status = lib().rsv_solve(A.h, M.h if M is not None else None, ctypes.byref(p), _ptr(b), _ptr(x),
                             ctypes.byref(st))
    _check(A.ctx, status, allow)
    d = st.as_dict()
    d["status"] = status
    if p.record_history:
        n = lib().rsv_solve_history(A.h, None, 0)
        import numpy as np
        h = np.zeros(n)
        lib().rsv_solve_history(A.h, h.ctypes.data, n)
        d["hist"] = h
    return d


class Net:
    def __init__(self, ctx: Context, c0=16, c1=32, c2=64, seed=0):
        arch = NetArch(3, c0, c1, c2)
        h = vp()
        _check(ctx, lib().rsv_net_create(ctx.h, ctypes.byref(arch), seed, ctypes.byref(h)))
        self.ctx, self.h = ctx, h

    @property
    def num_params(self):
        return lib().rsv_net_num_params(self.h)

    def get_params(self):
        import numpy as np
        out = np.zeros(self.num_params, np.float32)
        _check(self.ctx, lib().rsv_net_get_params(self.h, out.ctypes.data, out.size))
        return out

    def set_params(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(self.ctx, lib().rsv_net_set_params(self.h, w.ctypes.data, w.size))

    def save(self, path):
        _check(self.ctx, lib().rsv_net_save(self.h, path.encode()))

    def load(self, path):
        _check(self.ctx, lib().rsv_net_load(self.h, path.encode()))

    def forward(self, grid: Grid, r, lnk, z):
        _check(self.ctx, lib().rsv_net_forward(self.h, grid.h, _ptr(r), _ptr(lnk), _ptr(z)))
        return z

    def train_step(self, grid: Grid, nb, r, e, lnk, lr):
        loss = ctypes.c_float()
        _check(self.ctx, lib().rsv_net_train_step(self.h, grid.h, nb, _ptr(r), _ptr(e), _ptr(lnk), lr,
                                                  ctypes.byref(loss)))
        return loss.value

    def loss_grad(self, grid: Grid, nb, r, e, lnk):
        import numpy as np
        loss = ctypes.c_float()
        g = np.zeros(self.num_params, np.float32)
        _check(self.ctx, lib().rsv_net_loss_grad(self.h, grid.h, nb, _ptr(r), _ptr(e), _ptr(lnk),
                                                 ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def close(self):
        if self.h:
            lib().rsv_net_destroy(self.h)
            self.h = None


def conv3d(ctx: Context, dims, cin, cout, x, w, b, y):
    """One 3x3x3 layer: y[V][cout] (FP32) from x[V][cin] (BF16 bits, int16
    tensor), w[27][cin][cout] and b[cout] (FP32); all device tensors."""
    nx, ny, nz = dims
    _check(ctx, lib().rsv_conv3d(ctx.h, nx, ny, nz, cin, cout, _ptr(x), _ptr(w),
                                 _ptr(b) if b is not None else None, _ptr(y)))
    return y


def conv3d_bwd(ctx: Context, dims, cin, cout, x, w, dy, dx=None, dw=None, db=None):
    """Gradients of conv3d for dy[V][cout] (BF16 bits): dx, dw, db (FP32,
    device; any may be None)."""
    nx, ny, nz = dims
    opt = lambda t: _ptr(t) if t is not None else None  # noqa: E731
    _check(ctx, lib().rsv_conv3d_bwd(ctx.h, nx, ny, nz, cin, cout, _ptr(x), _ptr(w), _ptr(dy),
                                     opt(dx), opt(dw), opt(db)))
