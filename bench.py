#!/usr/bin/env python
"""Benchmark: time-to-solve of the 3x3-block 7-point reservoir Jacobian on one
MI355X, with the dominant kernel's achieved HBM bandwidth against the roofline
and the CPU oracle timed beside it.

Workload (default C5, the largest single-GPU configuration): 512x512x128
cells (100,663,296 unknowns), channelised permeability (bands of k = 1e3 in
k = 1 plus N(0,0.5) log noise), eight source cells, b = A x_true, x0 = 0,
tol 1e-8 on the recomputed FP64 relative residual.  One step = re-assemble
the block matrix from device blocks, then for each of the workload's three
preconditioner forms: setup + solve.  Forms: GMRES(30) + block ILU(0) with
FP64 factors (the headline time-to-solve), GMRES(30) + block ILU(0) with FP32
factors and sweeps, and FGMRES(30) + the learned U-Net preconditioner (BILU0
fallback), whose network is trained first on 64x64x32 systems (disjoint
seeds; training time reported apart) or loaded (--net).  BiCGSTAB + BILU0
and GMRES(30) + RAS(4x4x4) run once each after the timed steps.  Kernel
timings come from one more, untimed step with HIP events on the solver
stream.  --workload C2 gives the 128x128x64 workload with its own forms.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(nx, ny, nz):
    """Bytes each kernel must move per launch (stored blocks only, no padding,
    no re-reads), FP64."""
    c = nx * ny * nz
    N = 3 * c
    nl = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)   # lower (= upper) neighbour pairs
    nnzb = 2 * nl + c
    return {
        "nnzb": nnzb,
        "spmv": 72 * nnzb + 24 * N,            # A, x, y, plus the fused epilogue operand (b, rhat or s)
        "ilu_fwd": 72 * nl + 16 * N,            # L blocks, r in, y out
        "ilu_bwd": 72 * (nl + c) + 16 * N,      # U blocks + D^-1, y in, z out
        "ilu_apply": 72 * nnzb + 32 * N,
        "spmv_plain": 72 * nnzb + 16 * N,
        # FP32 factors: FP32 blocks and intermediate y, FP64 r in and z out
        "ilu_fwd_fp32": 36 * nl + 12 * N,
        "ilu_bwd_fp32": 36 * (nl + c) + 12 * N,
    }


def cpr_fpf_algorithmic_bytes(nx, ny, nz, fp32=False, coarse=128, pre=1, post=1):
    """Bytes the CPR-FPF kernels of one apply must move, the stage R's sweeps
    excluded (they are counted with the sweeps): the restricted residual
    (stored blocks of A, x, f and the weights, the pressure vector out), one
    multigrid V-cycle (every level's stored coefficients, b and x per colour
    sweep pair and per restriction, the coarsest level's inverse), the
    pressure correction folded into z (z_p read and written, e), the second
    residual (blocks, x, f, r out) and the final combination (z read and
    written, t)."""
    c = nx * ny * nz
    N = 3 * c
    ab = algorithmic_bytes(nx, ny, nz)
    wa = 36 if fp32 else 72
    wc = 4 if fp32 else 8
    resid0 = wa * ab["nnzb"] + 24 * N + 8 * c
    resid1 = wa * ab["nnzb"] + 24 * N
    prolong = 24 * c
    dims = [(nx, ny, nz)]
    while dims[-1][0] * dims[-1][1] * dims[-1][2] > coarse:
        dims.append(tuple((v + 1) // 2 if v > 1 else 1 for v in dims[-1]))
    mg = 0
    for l, (a, b_, c_) in enumerate(dims):
        n = a * b_ * c_
        if l == len(dims) - 1:
            mg += 8 * n * n + 16 * n
            break
        nzl = n + 2 * ((a - 1) * b_ * c_ + a * (b_ - 1) * c_ + a * b_ * (c_ - 1))
        nc = dims[l + 1][0] * dims[l + 1][1] * dims[l + 1][2]
        sweep = wc * nzl + 24 * n
        mg += pre * sweep + (wc * nzl + 16 * n + 8 * nc) + post * sweep + 8 * nc
    combine = 24 * N
    return {"resid": resid0 + resid1, "mg": mg, "prolong": prolong, "combine": combine,
            "apply": resid0 + resid1 + prolong + mg + combine, "levels": len(dims)}


def ras_algorithmic_bytes(nx, ny, nz, parts, ov):
    """Bytes of the local sweeps of RAS per launch: the stored blocks of every
    local matrix (couplings inside Omega_s) and the vector passes over every
    Omega_s cell, summed over the subdomains (padding of the boxes excluded)."""
    import numpy as np

    def starts(n, p):
        base, rem = divmod(n, p)
        return [b * base + min(b, rem) for b in range(p + 1)]

    xs, ys, zs = starts(nx, parts[0]), starts(ny, parts[1]), starts(nz, parts[2])
    c = nl = 0
    for sz in range(parts[2]):
        for sy in range(parts[1]):
            for sx in range(parts[0]):
                lo = [max(0, v - ov) for v in (xs[sx], ys[sy], zs[sz])]
                hi = [min(n, v + ov) for n, v in zip((nx, ny, nz), (xs[sx + 1], ys[sy + 1], zs[sz + 1]))]
                ax = [np.arange(a, b) for a, b in zip(lo, hi)]
                d = [np.maximum(0, np.maximum(core0 - a, a - (core1 - 1)))
                     for a, core0, core1 in zip(ax, (xs[sx], ys[sy], zs[sz]), (xs[sx + 1], ys[sy + 1], zs[sz + 1]))]
                inside = (d[0][:, None, None] + d[1][None, :, None] + d[2][None, None, :]) <= ov
                c += int(inside.sum())
                nl += int((inside[1:] & inside[:-1]).sum() + (inside[:, 1:] & inside[:, :-1]).sum()
                          + (inside[:, :, 1:] & inside[:, :, :-1]).sum())
    N = 3 * c
    return {"ilu_fwd": 72 * nl + 16 * N, "ilu_bwd": 72 * (nl + c) + 16 * N, "cells": c, "pairs": nl,
            "ilu_fwd_fp32": 36 * nl + 12 * N, "ilu_bwd_fp32": 36 * (nl + c) + 12 * N}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# per workload: the forms of one timed step (the first is the headline) and
# the forms run once after the timed steps
WORKLOAD_FORMS = {
    "C5": ("gmres_bilu0,gmres_bilu0_fp32", "gmres_bilu0_dcgs2,bicgstab_bilu0,gmres_ras64,gmres_ras64_iluk1,"
           "gmres_ras64_ilut,gmres_cpr_fpf,gmres_cpr_fpf_bilu0,bicgstab_cpr_fpf_bilu0,gmres_cpr_fpf_bilu0_fp32"),
    "C3": ("gmres_bilu0,gmres_bilu0_fp32", "gmres_ras64"),
    "C2": ("gmres_ras64,bicgstab_bilu0,gmres_bilu0,gmres_bilu0_fp32,gmres_ras64_fp32,gmres_ras64_dcgs2,"
           "gmres_bilu0_dcgs2,gmres_ras64_fp32_dcgs2,bicgstab_ras64,gmres_ras64_iluk1,gmres_cpr_fpf,"
           "gmres_cpr_fpf_bilu0,bicgstab_cpr_fpf_bilu0,gmres_cpr_fpf_fp32,gmres_cpr_fpf_bilu0_fp32,gmres_ras64_ilut", ""),
    "C4": ("gmres_bilu0,gmres_bilu0_fp32", ""),
    # (RAS over 4x4x4 boxes of 5x5x2 cells stagnates on the literal C1 matrix,
    # in the oracle as on the GPU: relative residual 2.8e-4 after 3000 steps)
    "C1": ("gmres_bilu0,gmres_bilu0_fp32", "bicgstab_bilu0"),
}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(cfg, Ao, bo, t_build, head_form, its_gpu, restart=30, full_limit_cells=4_000_000, k_sample=3):
    """The serial FP64 oracle on one host thread, on the same system.

    Up to full_limit_cells cells the whole solve of the headline form is
    timed.  Beyond that (the 512x512x128 workload: minutes of CPU time per
    solve), a bounded sample is timed -- the ILU(0) setup, one product, one
    preconditioner apply and a k_sample-step GMRES(30) run -- and the time to
    solve is projected for the GPU's iteration count with the per-step cost
    model t_M + t_A + c (j + 1) (apply, product, and c per basis vector of the
    two Gram-Schmidt passes at step j of a cycle; per cycle one residual
    product, one apply and one basis combination, c/4 per vector)."""
    import oracle as O
    method, pk = head_form
    host = {"cpu_model": cpu_model(), "host_logical_cores": os.cpu_count()}
    if cfg.ncell <= full_limit_cells:
        t1 = time.perf_counter()
        if pk.get("type") == 2:
            F = O.RAS(Ao, (cfg.nx, cfg.ny, cfg.nz), (pk["ras_px"], pk["ras_py"], pk["ras_pz"]), pk["ras_overlap"])
            what = "GMRES(30)+RAS(%dx%dx%d, overlap %d)" % (pk["ras_px"], pk["ras_py"], pk["ras_pz"], pk["ras_overlap"])
        else:
            F = O.ILU(Ao)
            what = "GMRES(30)+BILU0" if method == 0 else "BiCGSTAB+BILU0"
        if method == 1:
            ro = O.bicgstab(Ao, bo, pc=F, tol=1e-8, maxit=10000)
        else:
            ro = O.gmres(Ao, bo, pc=F, m=restart, tol=1e-8, maxit=10000)
        t2 = time.perf_counter()
        log(f"oracle: {t2 - t1:.2f}s ({ro['its']} its)")
        return {"value": round(t2 - t1, 3), "unit": "s", "cores": 1, "kind": "oracle",
                "sample": f"the whole {what} solve (setup and {ro['its']} iterations, relres {ro['relres']:.2e}) "
                          f"of the same system, serial FP64 C on one host thread; the oracle's matrix build "
                          f"from the blocks ({t_build:.1f}s) is not counted", **host}
    assert method == 0 and pk.get("type") == 1, "the projection models GMRES + BILU0"
    t1 = time.perf_counter()
    F = O.ILU(Ao)
    t_setup = time.perf_counter() - t1
    t1 = time.perf_counter()
    w = Ao.spmv(bo)
    t_A = time.perf_counter() - t1
    t1 = time.perf_counter()
    F.apply(w)
    t_M = time.perf_counter() - t1
    t1 = time.perf_counter()
    ro = O.gmres(Ao, bo, pc=F, m=restart, tol=0.0, maxit=k_sample)
    T_k = time.perf_counter() - t1
    # T_k = t_A + sum_{j<k}(t_M + t_A + c(j+1)) + (t_M + c k/4) + t_A
    k = k_sample
    c = max(0.0, (T_k - 2 * t_A - t_M - k * (t_M + t_A)) / (k * (k + 1) / 2 + k / 4))
    proj = t_setup + t_A
    left = its_gpu
    while left > 0:
        L = min(restart, left)
        proj += sum(t_M + t_A + c * (j + 1) for j in range(L)) + t_M + c * L / 4 + t_A
        left -= L
    sample_s = t_setup + t_A + t_M + T_k
    log(f"oracle sample: setup {t_setup:.1f}s, product {t_A:.2f}s, apply {t_M:.2f}s, "
        f"{k_sample} GMRES steps {T_k:.1f}s (c = {c:.3f}s per basis vector); projection {proj:.1f}s")
    return {"value": round(proj, 2), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"projected time to solve for {its_gpu} GMRES(30)+BILU0 steps from a timed sample on "
                       f"the same system ({sample_s:.1f}s of CPU work): ILU(0) setup {t_setup:.2f}s, one block "
                       f"product {t_A:.3f}s, one ILU(0) apply {t_M:.3f}s, and a {k_sample}-step GMRES(30) run "
                       f"{T_k:.2f}s giving {c:.4f}s per basis vector of the two Gram-Schmidt passes; per step "
                       f"t_M + t_A + c(j+1), per cycle one residual product, one apply and c/4 per vector of the "
                       f"basis combination; serial FP64 C on one host thread, the oracle's matrix build from "
                       f"the blocks ({t_build:.1f}s) not counted"),
            "sample_s": round(sample_s, 2), "setup_s": round(t_setup, 3), "product_s": round(t_A, 4),
            "apply_s": round(t_M, 4), "gmres_steps": k_sample, "gmres_steps_s": round(T_k, 3),
            "per_basis_vector_s": round(c, 5), **host}


def hsfc_measure(rsv, ctx, g, dims, levels, nparts, reps=5, cpu=True):
    """The Hilbert-curve partition of the grid (keys of the cell centroids,
    the equal-count cut, the partition quality), timed with events around
    each library call after one untimed pass; the oracle's keys and partition
    of the same grid timed on one host thread beside it.  Algorithmic bytes:
    keys write 8 B per cell; each 8-bit pass of the radix sort reads the keys
    for its histogram (8 B), then reads key and index (12 B, 8 B on the first
    pass) and writes them (12 B); the cut reads the indices and writes the
    parts (8 B)."""
    import numpy as np
    import torch
    n = g.ncell
    keys = torch.zeros(n, dtype=torch.int64, device="cuda")
    part = torch.zeros(n, dtype=torch.int32, device="cuda")
    passes = (3 * levels + 7) // 8
    t = {"keys": [], "partition": [], "quality": []}
    for r in range(reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        g.hsfc_keys(levels, keys)
        e[1].record()
        rsv.hsfc_partition(ctx, keys, levels, nparts, part)
        e[2].record()
        q, _ = g.partition_quality(part, nparts)
        e[3].record()
        torch.cuda.synchronize()
        if r > 0:
            t["keys"].append(e[0].elapsed_time(e[1]) * 1e-3)
            t["partition"].append(e[1].elapsed_time(e[2]) * 1e-3)
            t["quality"].append(e[2].elapsed_time(e[3]) * 1e-3)
    med = {k: float(np.median(v)) for k, v in t.items()}
    part_bytes = n * (passes * 8 + (passes * 24 - 4) + 8)
    out = {"workload": f"Hilbert-curve partition of the {dims[0]}x{dims[1]}x{dims[2]} grid into {nparts} parts, "
                       f"{levels} levels ({passes} radix passes)",
           "keys_s": round(med["keys"], 6), "partition_s": round(med["partition"], 6),
           "quality_s": round(med["quality"], 6),
           "cells_per_s": round(n / (med["keys"] + med["partition"]), 1),
           "quality": {"load_imbalance": q[0], "max_local_surface_index": q[1], "global_surface_index": q[2],
                       "average_surface_index": q[3], "max_connectivity": int(q[4])},
           "roofline": {"bound": "hbm", "kernel": "partition (histograms, scan, scatters, cut)",
                        "achieved": round(part_bytes / med["partition"] / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(part_bytes / med["partition"] / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": None, "algorithmic_bytes": part_bytes}}
    del keys, part
    if cpu:
        from oracle import hsfc as H
        t0 = time.perf_counter()
        kh = H.grid_keys(dims, levels)
        t1 = time.perf_counter()
        H.partition(kh, nparts)
        t2 = time.perf_counter()
        out["cpu_baseline"] = {"value": round(n / (t2 - t0), 1), "unit": "cells/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's keys ({t1 - t0:.2f}s) and qsort-based cut ({t2 - t1:.2f}s) "
                                         f"of the whole grid, one host thread"}
    return out


def poisson_measure(rsv, ctx, dims, parts, its=90, reps=3, cpu=True):
    """The paper's Poisson Equation example at one GPU's size: the scalar
    7-point Laplacian on dims cells, b = A x_true, GMRES(30) with RAS
    (parts subdomains -- about the paper's cells per core at 4096 cores --
    overlap one, ILU(0) on every subdomain) run for a fixed `its` iterations
    as the paper runs 90; the median of `reps` timed runs after one untimed,
    then one untimed run with kernel events.  The oracle's cost per iteration
    is taken on a sample of four subdomains of the same shape (a 2x2x1 box of
    them), projected to the whole grid by the cell count."""
    import numpy as np
    import torch
    from paper_1602_05901_amd import inputs as I
    cfg = I.GenConfig(*dims, I.LNK_IID, 0.0, 0.0, 0.0, 0, 1e3, 1.0, 0)
    t0 = time.time()
    C = I.poisson(cfg)
    xt = I.x_true_scalar(cfg)
    log(f"poisson: generated {dims} in {time.time() - t0:.1f}s")
    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, torch.from_numpy(C).cuda(), scalar=True)
    del C
    xtd = torch.from_numpy(xt).cuda()
    b = torch.zeros_like(xtd)
    A.spmv(xtd, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = rsv.Precond(A, type=rsv.PC_RAS, ras_px=parts[0], ras_py=parts[1], ras_pz=parts[2], ras_overlap=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    times, st = [], None
    for r in range(reps + 2):
        x = torch.zeros_like(b)
        prof = r == reps + 1
        if prof:
            ctx.profile(True, classes=("spmv", "ras", "ortho"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = rsv.solve(A, M, b, x, method=rsv.GMRES, restart=30, tol=0.0, maxit=its)
        torch.cuda.synchronize()
        if prof:
            kr = ctx.profile_read()
            ctx.profile(False)
        elif r > 0:
            times.append(time.perf_counter() - t0)
    err = float(torch.linalg.norm(x - xtd) / torch.linalg.norm(xtd))
    n = cfg.ncell
    solve_s = float(np.median(times))
    nnz = 7 * n - 2 * (dims[1] * dims[2] + dims[0] * dims[2] + dims[0] * dims[1])
    spmv_bytes = 8 * nnz + 16 * n
    kern = {k: {"avg_us": 1e3 * kr[k][0] / kr[k][1], "launches": kr[k][1]} for k in ("spmv", "ras", "ortho")
            if kr[k][1]}
    if "spmv" in kern:
        kern["spmv"]["GBps"] = spmv_bytes / (kern["spmv"]["avg_us"] * 1e-6) / 1e9
    ras_bytes = M.apply_bytes
    if "ras" in kern and ras_bytes > 0:
        # the library's own count of one apply: per Omega_s cell its factors
        # and three vector passes, per grid cell the result, per x-chunk its ids
        gbps = ras_bytes / (kern["ras"]["avg_us"] * 1e-6) / 1e9
        kern["ras"].update({"algorithmic_bytes": ras_bytes, "GBps": round(gbps, 1),
                            "frac": round(gbps / HBM_PEAK_GBS, 4)})
    out = {"workload": f"scalar 7-point Laplacian {dims[0]}x{dims[1]}x{dims[2]} ({n} unknowns), GMRES(30) + RAS "
                       f"({parts[0]}x{parts[1]}x{parts[2]} subdomains of about {n // (parts[0] * parts[1] * parts[2])} "
                       f"cells, overlap 1, ILU(0)), {its} iterations",
           "setup_s": round(setup_s, 4), "solve_s": round(solve_s, 4), "its": st["its"],
           "s_per_iteration": round(solve_s / its, 6), "relres_after": st["final_relres"], "err_vs_xtrue": err,
           "unknown_iterations_per_s": round(n * its / solve_s, 1), "kernels": kern,
           "paper_context": {"workload": "Poisson equation, 3e9 cells, GMRES(30) + RAS(overlap 1, ILU(0)), 90 iterations",
                             "hardware": "IBM Blue Gene/Q", "solve_s_512_cores": 606.33,
                             "solve_s_4096_cores": 80.30, "s_per_iteration_4096_cores": round(80.30 / 90, 3),
                             "unknown_iterations_per_s_4096_cores": round(3e9 * 90 / 80.30, 1),
                             "note": "solve = overall - gridding - building - assemble of the table's row"}}
    M.close(); A.close(); g.close()
    del b, xtd
    if cpu:
        from oracle import scalar as S
        sx = -(-dims[0] // parts[0]) * 2
        sy = -(-dims[1] // parts[1]) * 2
        sz = -(-dims[2] // parts[2])
        sc = I.GenConfig(sx, sy, sz, I.LNK_IID, 0.0, 0.0, 0.0, 0, 1e3, 1.0, 0)
        Ao = S.CSR(sx, sy, sz, I.poisson(sc))
        bo = Ao.spmv(I.x_true_scalar(sc))
        t0 = time.perf_counter()
        R = S.RAS(Ao, (sx, sy, sz), (2, 2, 1), 1)
        t1 = time.perf_counter()
        k = 5
        S.gmres(Ao, bo, pc=R, m=30, tol=0.0, maxit=k)
        t2 = time.perf_counter()
        per_cell_it = (t2 - t1) / k / sc.ncell
        out["cpu_baseline"] = {"value": round(per_cell_it * n * its, 2), "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's GMRES(30) + RAS on a {sx}x{sy}x{sz} grid of four subdomains "
                                         f"of the same shape ({k} iterations in {t2 - t1:.2f}s after a {t1 - t0:.2f}s "
                                         f"setup), scaled by cells and to {its} iterations; one host thread"}
    return out


# (grid, input channels, output channels) of the network's layers at the
# 512x512x128 workload: level 0 full resolution, level 1 half, level 2 quarter
CONV_LAYERS = [((512, 512, 128), 4, 16), ((512, 512, 128), 16, 16), ((512, 512, 128), 32, 16),
               ((256, 256, 64), 16, 32), ((256, 256, 64), 32, 32), ((128, 128, 32), 32, 64),
               ((128, 128, 32), 64, 64), ((256, 256, 64), 64, 32)]


def conv_layers(rsv, torch, reps=5):
    """Time single layers (`rsv_conv3d`: BF16 in, FP32 out, bias, weight
    packing included): one untimed launch, then the mean of `reps`; prints
    one JSON line."""
    ctx = rsv.Context(0)
    out = []
    for dims, cin, cout in CONV_LAYERS:
        V = dims[0] * dims[1] * dims[2]
        gen = torch.Generator(device="cuda").manual_seed(cin * 100 + cout)
        # BF16 bit patterns of finite values in [0, 0.5)
        x = torch.randint(0, 0x3F00, (V * cin,), dtype=torch.int16, device="cuda", generator=gen)
        w = torch.randn(27 * cin * cout, dtype=torch.float32, device="cuda", generator=gen) * 0.1
        b = torch.zeros(cout, dtype=torch.float32, device="cuda")
        y = torch.zeros(V * cout, dtype=torch.float32, device="cuda")
        rsv.conv3d(ctx, dims, cin, cout, x, w, b, y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            rsv.conv3d(ctx, dims, cin, cout, x, w, b, y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / reps * 1e3
        flop = 2 * 27 * cin * cout * V
        out.append({"grid": list(dims), "cin": cin, "cout": cout, "ms": round(ms, 4),
                    "TFLOPs": round(flop / ms / 1e9, 1), "of_bf16_peak": round(flop / ms / 1e9 / 2500.0, 4)})
        log(f"conv {dims} {cin}->{cout}: {ms:.3f} ms")
        del x, y
    print(json.dumps({"conv_layers": out}), flush=True)
    ctx.close()


def copy_probe(torch, dev):
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: 1073741824 bytes read, 1073741824 bytes written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C5")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default=None, help="forms of a timed step, comma separated (first = headline)")
    ap.add_argument("--extra-forms", default=None, help="forms run once after the timed steps")
    ap.add_argument("--net", default=None, help="trained U-Net weights for the learned form")
    ap.add_argument("--learned-steps", type=int, default=1500,
                    help="without --net: Adam steps of training on C4 systems before the timed steps (0: no learned form)")
    ap.add_argument("--learned-seeds", default="1000-1015")
    ap.add_argument("--theta", type=float, default=0.9, help="the learned form's fallback threshold")
    ap.add_argument("--no-profile", action="store_true", help="skip the untimed kernel-timing step")
    ap.add_argument("--hsfc-parts", type=int, default=64,
                    help="parts of the Hilbert-curve partition of the workload's grid timed after the solves (0: skip)")
    ap.add_argument("--poisson", default="512,512,512:6,6,5",
                    help="grid:subdomains of the scalar Poisson run after the solves (empty: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with one device-to-device copy of 1 GiB (calibrates HBM byte counters)")
    ap.add_argument("--conv-layers", action="store_true",
                    help="only time single 3x3x3 convolution layers at the learned form's sizes and print them")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1602_05901_amd import inputs as I
    from paper_1602_05901_amd import rsv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.conv_layers:
        conv_layers(rsv, torch)
        if args.copy_probe:
            copy_probe(torch, dev)
        return
    wl = args.workload.upper()
    cfg = I.preset(wl, seed=args.seed)
    dforms, dextra = WORKLOAD_FORMS.get(wl, ("gmres_bilu0", ""))
    forms = [f for f in (args.forms if args.forms is not None else dforms).split(",") if f]
    extra = [f for f in (args.extra_forms if args.extra_forms is not None else dextra).split(",") if f]
    t0 = time.time()
    lnk = I.lnk(cfg)
    B = I.blocks(cfg, lnk)
    xt = I.x_true(cfg)
    log(f"generated {wl} {cfg.nx}x{cfg.ny}x{cfg.nz} in {time.time() - t0:.1f}s")
    Bd = torch.from_numpy(B).to(dev)
    xtd = torch.from_numpy(xt).to(dev)
    ctx = rsv.Context(0)
    g = rsv.Grid(ctx, cfg.nx, cfg.ny, cfg.nz)
    A = rsv.Matrix(g, Bd)
    # the host-buffer path of the boundary (blocks in host memory, copied over
    # PCIe and laid out by the library): timed once, never part of `value`
    torch.cuda.synchronize()
    th = time.perf_counter()
    Ah = rsv.Matrix(g, B)
    torch.cuda.synchronize()
    host_assemble_s = time.perf_counter() - th
    Ah.close()
    b = torch.zeros_like(xtd)
    A.spmv(xtd, b)          # manufactured right-hand side, on the GPU
    torch.cuda.synchronize()

    ras = dict(ras_px=4, ras_py=4, ras_pz=4, ras_overlap=1)
    forms_all = {
        "bicgstab_bilu0": (rsv.BICGSTAB, dict(type=rsv.PC_BILU0)),
        "gmres_ras64": (rsv.GMRES, dict(type=rsv.PC_RAS, **ras)),
        "gmres_ras64_fp32": (rsv.GMRES, dict(type=rsv.PC_RAS, precision=rsv.FP32, **ras)),
        "bicgstab_ras64": (rsv.BICGSTAB, dict(type=rsv.PC_RAS, **ras)),
        "gmres_bilu0": (rsv.GMRES, dict(type=rsv.PC_BILU0)),
        "gmres_bilu0_fp32": (rsv.GMRES, dict(type=rsv.PC_BILU0, precision=rsv.FP32)),
        # RAS with ILU(1) local solvers (the RAS parameters' iluk_level 1)
        "gmres_ras64_iluk1": (rsv.GMRES, dict(type=rsv.PC_RAS, iluk_level=1, **ras)),
        # RAS with ILUT(-1, 1e-3) local solvers (the RAS parameters' ILUT defaults)
        "gmres_ras64_ilut": (rsv.GMRES, dict(type=rsv.PC_RAS, local_solver=rsv.LOCAL_ILUT, **ras)),
        # CPR-FPF two-stage preconditioners (stage R = RAS(4x4x4) or BILU0,
        # pressure stage = one aggregation-multigrid V-cycle, no decoupling)
        "gmres_cpr_fpf": (rsv.GMRES, dict(type=rsv.PC_CPR, cpr_stage=rsv.PC_RAS, **ras)),
        "gmres_cpr_fpf_bilu0": (rsv.GMRES, dict(type=rsv.PC_CPR, cpr_stage=rsv.PC_BILU0)),
        "bicgstab_cpr_fpf_bilu0": (rsv.BICGSTAB, dict(type=rsv.PC_CPR, cpr_stage=rsv.PC_BILU0)),
        # the FP32 form of CPR-FPF: FP32 sweeps, FP32 copies of A and of the level operators
        "gmres_cpr_fpf_fp32": (rsv.GMRES, dict(type=rsv.PC_CPR, cpr_stage=rsv.PC_RAS, precision=rsv.FP32, **ras)),
        "gmres_cpr_fpf_bilu0_fp32": (rsv.GMRES, dict(type=rsv.PC_CPR, cpr_stage=rsv.PC_BILU0, precision=rsv.FP32)),
    }
    forms_all["gmres_cpr_fpf_bilu0_fp32_dcgs2"] = forms_all["gmres_cpr_fpf_bilu0_fp32"]
    # the same GMRES forms with the delayed second Gram-Schmidt pass
    for f in ("gmres_ras64", "gmres_bilu0", "gmres_ras64_fp32"):
        forms_all[f + "_dcgs2"] = forms_all[f]
    net = None
    training = None
    if args.net or args.learned_steps > 0:
        net = rsv.Net(ctx)
        if args.net:
            net.load(args.net)
        else:
            # train on 64x64x32 systems (disjoint seeds), reported apart from the solves
            from paper_1602_05901_amd import train as T
            t0 = time.perf_counter()
            a, z = (int(v) for v in args.learned_seeds.split("-"))
            data = []
            for sd in range(a, z + 1):
                sy = T.System(ctx, I.preset("C4", seed=sd))
                R, E, _ = T.harvest(ctx, sy)
                data.append((sy.g, R, E, sy.lnk, sy))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            losses = T.train(ctx, net, [d[:4] for d in data], args.learned_steps, batch=8, lr=1e-3, seed=0)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            training = {"workload": "C4 64x64x32", "seeds": args.learned_seeds,
                        "pairs": int(sum(d[1].shape[0] for d in data)), "harvest_s": round(t1 - t0, 3),
                        "steps": args.learned_steps, "batch": 8, "train_s": round(t2 - t1, 3),
                        "loss_first": losses[0], "loss_last": float(np.mean(losses[-50:]))}
            log(f"trained the network: {training}")
            for d in data:
                d[4].close()
            del data
        lnk32 = torch.from_numpy(lnk.astype(np.float32)).to(dev)
        forms_all["fgmres_learned"] = (rsv.FGMRES, dict(type=rsv.PC_LEARNED, net=net, lnk=lnk32, theta=args.theta))
        forms.append("fgmres_learned")

    hbm_peak = [0]   # device memory in use (all allocations, torch and the library) after each solve
    apply_bytes = {}  # per form: the library's algorithmic bytes of one apply (level-scheduled solvers)

    def run_form(name, profile=False, keep_x=False):
        method, pkw = forms_all[name]
        t1 = time.perf_counter()
        M = rsv.Precond(A, **pkw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x = torch.zeros_like(b)
        if profile:
            ctx.profile(True, classes=("spmv", "ilu_fwd", "ilu_bwd", "ortho", "cpr", "ras"))
        st = rsv.solve(A, M, b, x, method=method, restart=30, tol=1e-8, maxit=10000,
                       ortho=(rsv.DCGS2 if name.endswith("_dcgs2") else rsv.CGS2))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        kern = None
        if profile:
            kern = ctx.profile_read()
            ctx.profile(False)
        apply_bytes[name] = M.apply_bytes
        free_b, total_b = torch.cuda.mem_get_info()
        hbm_peak[0] = max(hbm_peak[0], total_b - free_b)
        err = float(torch.linalg.norm(x - xtd) / torch.linalg.norm(xtd))
        out = {"setup_s": t2 - t1, "solve_s": t3 - t2, "its": st["its"], "relres": st["final_relres"],
               "status": st["status"], "err_vs_xtrue": err, "fallbacks": st["fallbacks"]}
        M.close()
        assert st["status"] == rsv.OK and st["final_relres"] <= 1e-8, (name, st)
        return out, kern, (x if keep_x else None)

    def step():
        out = {}
        torch.cuda.synchronize()
        ta = time.perf_counter()
        A.update(Bd)
        torch.cuda.synchronize()
        out["assemble_s"] = time.perf_counter() - ta
        for name in forms:
            out[name] = run_form(name)[0]
        return out

    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: " + ", ".join(f"{k} {r[k]['solve_s'] * 1e3:.1f}ms/{r[k]['its']}its" for k in forms))
    torch.cuda.synchronize()
    res = []
    tt = time.perf_counter()
    for s in range(args.steps):
        r = step()
        res.append(r)
        log(f"step {s}: " + ", ".join(f"{k} {r[k]['solve_s'] * 1e3:.1f}ms/{r[k]['its']}its" for k in forms))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tt

    def med(key, sub):
        return float(np.median([r[key][sub] for r in res]))

    head = forms[0]
    summary = {f: {"solve_s": med(f, "solve_s"), "setup_s": med(f, "setup_s"), "its": res[-1][f]["its"],
                   "relres": res[-1][f]["relres"], "err_vs_xtrue": res[-1][f]["err_vs_xtrue"],
                   "fallbacks": res[-1][f]["fallbacks"]} for f in forms}

    # -------- after the timed steps: kernel timing, the FP64 oracle's view of each
    # result, and the forms run once
    ab_global = algorithmic_bytes(cfg.nx, cfg.ny, cfg.nz)
    ab_ras = None
    kernels_by_form = {}
    xs = {}
    if not args.no_profile:
        for f in forms:
            o, kern, x = run_form(f, profile=True, keep_x=True)
            kernels_by_form[f] = kern
            xs[f] = x.cpu().numpy()
            del x
    solves_once = {}
    for f in extra:
        o, kern, x = run_form(f, profile=not args.no_profile, keep_x=True)
        solves_once[f] = o
        kernels_by_form[f] = kern
        xs[f] = x.cpu().numpy()
        del x
        log(f"{f}: {o['solve_s'] * 1e3:.1f}ms/{o['its']}its")

    def kernel_table(form):
        nonlocal ab_ras
        kr = kernels_by_form[form]
        kms = {k: kr[k][0] for k in rsv.K_NAMES}
        kcnt = {k: kr[k][1] for k in rsv.K_NAMES}
        ab = dict(ab_global)
        if forms_all[form][0] != rsv.BICGSTAB:
            # GMRES products (y = A z with ||y||^2) read no third vector; the few
            # residual launches per solve that do read b are counted the same
            ab["spmv"] = ab_global["spmv_plain"]
        pk = forms_all[form][1]
        if pk.get("precision") == rsv.FP32 and pk.get("type") in (rsv.PC_BILU0, rsv.PC_CPR) and \
                pk.get("cpr_stage", rsv.PC_BILU0) == rsv.PC_BILU0:
            ab["ilu_fwd"], ab["ilu_bwd"] = ab_global["ilu_fwd_fp32"], ab_global["ilu_bwd_fp32"]
        if pk.get("type") == rsv.PC_RAS or (pk.get("type") == rsv.PC_CPR and pk.get("cpr_stage") == rsv.PC_RAS):
            # the sweeps of this form are the local RAS sweeps
            ab_ras = ras_algorithmic_bytes(cfg.nx, cfg.ny, cfg.nz, (pk["ras_px"], pk["ras_py"], pk["ras_pz"]),
                                           pk["ras_overlap"])
            sfx = "_fp32" if pk.get("precision") == rsv.FP32 else ""
            ab["ilu_fwd"], ab["ilu_bwd"] = ab_ras["ilu_fwd" + sfx], ab_ras["ilu_bwd" + sfx]
        tab = {k: {"avg_us": 1e3 * kms[k] / kcnt[k], "launches": kcnt[k], "total_ms": kms[k],
                   "GBps": (ab[k] / (kms[k] / kcnt[k] * 1e-3) / 1e9) if k in ab and k != "ilu_apply" else None}
               for k in rsv.K_NAMES if kcnt[k] > 0}
        if kcnt["ras"] > 0 and apply_bytes.get(form, -1) > 0:
            # the level-scheduled local solvers (ILU(k), ILUT): one launch per apply
            gb = apply_bytes[form] / (kms["ras"] / kcnt["ras"] * 1e-3) / 1e9
            tab["ras"].update({"algorithmic_bytes_per_apply": apply_bytes[form], "GBps": gb,
                               "frac": round(gb / HBM_PEAK_GBS, 4)})
        if pk.get("type") == rsv.PC_CPR and kcnt["cpr"] > 0:
            # CPR-FPF records five timed scopes per apply: the restricted
            # residual, the V-cycle, the correction of z, the residual and the
            # combination
            cb = cpr_fpf_algorithmic_bytes(cfg.nx, cfg.ny, cfg.nz, fp32=pk.get("precision") == rsv.FP32)
            napply = kcnt["cpr"] // 5
            ms_apply = kms["cpr"] / max(napply, 1)
            tab["cpr"].update({"applies": napply, "ms_per_apply": ms_apply,
                               "algorithmic_bytes_per_apply": cb["apply"], "mg_levels": cb["levels"],
                               "GBps": cb["apply"] / (ms_apply * 1e-3) / 1e9,
                               "frac": round(cb["apply"] / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        return kms, kcnt, ab, tab

    roofline = None
    kernels = {}
    if kernels_by_form:
        kms, kcnt, ab, kernels_head = kernel_table(head)
        kernels[head] = kernels_head
        for f in kernels_by_form:
            if f != head:
                kernels[f] = kernel_table(f)[3]
        cand = [k for k in ("spmv", "ilu_fwd", "ilu_bwd") if kcnt[k] > 0]
        dom = max(cand, key=lambda k: kms[k])
        avg_ms = kms[dom] / kcnt[dom]
        achieved = ab[dom] / (avg_ms * 1e-3) / 1e9
        traffic = None
        tpath = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tpath):
            try:
                tj = json.load(open(tpath))
                traffic = tj["workloads"][wl]["forms"][head]["kernels"][dom]["bytes_per_launch"]
            except Exception:  # noqa: BLE001
                traffic = None
        roofline = {"bound": "hbm", "kernel": dom, "form": head, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "algorithmic_bytes_per_launch": ab[dom],
                    "avg_launch_us": round(avg_ms * 1e3, 2),
                    "share_of_solve_kernel_time": {k: round(kms[k] / max(sum(kms.values()), 1e-30), 3)
                                                   for k in ("spmv", "ilu_fwd", "ilu_bwd", "ortho")},
                    "timing": "HIP events on the solver stream in one untimed solve after the timed steps"}

    # the FP64 oracle's product recomputes the relative residual of every
    # returned solution; each solution is also compared with the FP64 one
    oracle_view = None
    Ao = bo = None
    t_build = 0.0
    if xs or not args.no_cpu_baseline:
        import oracle as O
        t0 = time.perf_counter()
        Ao = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, B)
        bo = Ao.spmv(xt)
        t_build = time.perf_counter() - t0
    if xs:
        t0 = time.perf_counter()
        nbo = float(np.linalg.norm(bo))
        ref = xs.get("gmres_bilu0", xs[head])
        oracle_view = {}
        for f, x in xs.items():
            oracle_view[f] = {"relres_by_oracle_spmv": float(np.linalg.norm(bo - Ao.spmv(x)) / nbo),
                              "err_vs_fp64_gmres_bilu0_solution": float(np.linalg.norm(x - ref) / np.linalg.norm(ref))}
        log(f"oracle residual check in {time.perf_counter() - t0:.1f}s: {oracle_view}")
    xs.clear()

    cpu = None
    if not args.no_cpu_baseline:
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        cpu = oracle_baseline(cfg, Ao, bo, t_build, forms_all[head], summary[head]["its"])
    del Ao, bo

    hsfc = None
    if args.hsfc_parts > 0:
        L = max(cfg.nx, cfg.ny, cfg.nz)
        levels = max(1, (L - 1).bit_length())      # enough levels to give every cell its own key
        hsfc = hsfc_measure(rsv, ctx, g, (cfg.nx, cfg.ny, cfg.nz), levels, args.hsfc_parts,
                            cpu=not args.no_cpu_baseline)
        log(f"hsfc: {hsfc}")

    # the runtime's device-to-device copy rate beside the vendor peak, for context
    # (1 GiB read + 1 GiB written, median of five, outside the timed steps)
    csrc = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    ct = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cdst.copy_(csrc)
        e1.record()
        torch.cuda.synchronize()
        ct.append(e0.elapsed_time(e1) * 1e-3)
    copy_GBps = round(2 * csrc.numel() * 8 / float(np.median(ct)) / 1e9, 1)
    del csrc, cdst
    if roofline is not None:
        roofline["d2d_copy_GBps"] = copy_GBps

    poisson = None
    if args.poisson:
        A_keep_bytes = A.device_bytes
        A.close()                                 # the block matrix and its workspace make room
        pd, pp = args.poisson.split(":")
        poisson = poisson_measure(rsv, ctx, tuple(int(v) for v in pd.split(",")), tuple(int(v) for v in pp.split(",")),
                                  cpu=not args.no_cpu_baseline)
        log(f"poisson: {poisson}")
    else:
        A_keep_bytes = A.device_bytes

    value = summary[head]["solve_s"]
    line = {
        "metric": "time-to-solve to 1e-8 FP64 rel. residual (s), SpMV/ILU HBM GB/s; learned/FP32 vs plain",
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl} {cfg.nx}x{cfg.ny}x{cfg.nz} 3x3-block 7-point, headline {head}, tol 1e-8",
                   "unknowns": 3 * cfg.ncell, "forms": forms, "forms_once": extra, "seed": args.seed,
                   "step": "re-assemble from device blocks, then setup + solve of every form in forms"},
        "solves": summary,
        "solves_once": solves_once,
        "vs_plain_gmres_bilu0": ({f: round(summary[f]["solve_s"] / summary["gmres_bilu0"]["solve_s"], 3) for f in forms}
                                 if "gmres_bilu0" in summary else None),
        "oracle_view": oracle_view,
        "learned_training": training,
        # unknowns x iterations per second of the headline solve, beside the paper's
        # closest published figure (scalar Poisson on a CPU cluster): context only
        "unknown_iterations_per_s": round(3 * cfg.ncell * summary[head]["its"] / value, 1),
        "paper_context": {"workload": "scalar 7-point Poisson, 3e9 unknowns, GMRES(30) + RAS(overlap 1, ILU(0)), "
                                      "90 iterations (Poisson Equation example)",
                          "hardware": "IBM Blue Gene/Q, 512 cores (PowerPC A2)",
                          "solve_s": 606.33, "unknown_iterations_per_s": round(3e9 * 90 / 606.33, 1),
                          "note": "solve time = overall - gridding - building - assemble of its 512-core row"},
        "kernels": kernels,
        "ras_local": ab_ras,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hsfc_partition": hsfc,
        "poisson_ras": poisson,
        "assemble_from_host_s": round(host_assemble_s, 4),
        "assemble_from_host_GBps": round(B.nbytes / host_assemble_s / 1e9, 2),
        "device_bytes": A_keep_bytes,
        "hbm_used_bytes": int(hbm_peak[0]),
        "hbm_total_bytes": int(torch.cuda.mem_get_info()[1]),
        "device": ctx.device_info(),
    }
    print(json.dumps(line), flush=True)
    if args.copy_probe:
        copy_probe(torch, dev)
    if not args.poisson:
        A.close()
    g.close(); ctx.close()


if __name__ == "__main__":
    main()
