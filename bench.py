#!/usr/bin/env python
"""Benchmark: time-to-solve of the 3x3-block 7-point reservoir Jacobian on one
MI355X, with the dominant kernel's achieved HBM bandwidth against the roofline
and the CPU oracle timed beside it.

Workload (default C2): 128x128x64 cells (3,145,728 unknowns), layered
log-normal permeability (layer mean ~ N(0,1.5), cell noise ~ N(0,2)), four
source cells, b = A x_true, x0 = 0, tol 1e-8 on the recomputed FP64 relative
residual.  One step = assemble the block matrix, then for each solver form:
preconditioner setup + solve.  Forms: GMRES(30) + RAS(4x4x4 subdomains,
overlap 1, ILU(0) local solves: the paper's own solver configuration, the
headline time-to-solve), BiCGSTAB + BILU0,
GMRES(30) + BILU0 with FP64 factors, GMRES(30) + BILU0 with FP32 factors,
GMRES(30) + RAS with FP32 local factors,
and FGMRES(30) + the learned U-Net preconditioner (BILU0 fallback), whose
network is trained first on C4-shaped systems (64x64x32, disjoint seeds;
training time reported apart) or loaded (--net).

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
    }


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
    return {"ilu_fwd": 72 * nl + 16 * N, "ilu_bwd": 72 * (nl + c) + 16 * N, "cells": c, "pairs": nl}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="gmres_ras64,bicgstab_bilu0,gmres_bilu0,gmres_bilu0_fp32,gmres_ras64_fp32,"
                                          "gmres_ras64_dcgs2,gmres_bilu0_dcgs2,gmres_ras64_fp32_dcgs2,bicgstab_ras64")
    ap.add_argument("--net", default=None, help="trained U-Net weights for the learned form")
    ap.add_argument("--learned-steps", type=int, default=1500,
                    help="without --net: Adam steps of training on C4 systems before the timed steps (0: no learned form)")
    ap.add_argument("--learned-seeds", default="1000-1015")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with one device-to-device copy of 1 GiB (calibrates HBM byte counters)")
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
    cfg = I.preset(args.workload, seed=args.seed)
    t0 = time.time()
    lnk = I.lnk(cfg)
    B = I.blocks(cfg, lnk)
    xt = I.x_true(cfg)
    log(f"generated {args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} in {time.time() - t0:.1f}s")
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

    forms_all = {
        "bicgstab_bilu0": (rsv.BICGSTAB, dict(type=rsv.PC_BILU0)),
        "gmres_ras64": (rsv.GMRES, dict(type=rsv.PC_RAS, ras_px=4, ras_py=4, ras_pz=4, ras_overlap=1)),
        "gmres_ras64_fp32": (rsv.GMRES, dict(type=rsv.PC_RAS, ras_px=4, ras_py=4, ras_pz=4, ras_overlap=1,
                                              precision=rsv.FP32)),
        "bicgstab_ras64": (rsv.BICGSTAB, dict(type=rsv.PC_RAS, ras_px=4, ras_py=4, ras_pz=4, ras_overlap=1)),
        "gmres_bilu0": (rsv.GMRES, dict(type=rsv.PC_BILU0)),
        "gmres_bilu0_fp32": (rsv.GMRES, dict(type=rsv.PC_BILU0, precision=rsv.FP32)),
    }
    # the same GMRES forms with the delayed second Gram-Schmidt pass
    for f in ("gmres_ras64", "gmres_bilu0", "gmres_ras64_fp32"):
        forms_all[f + "_dcgs2"] = forms_all[f]
    forms = [f for f in args.forms.split(",") if f]
    net = None
    lnk32 = None
    training = None
    if args.net or args.learned_steps > 0:
        net = rsv.Net(ctx)
        if args.net:
            net.load(args.net)
        else:
            # train on C4-shaped systems (disjoint seeds), reported apart from the solves
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
        forms_all["fgmres_learned"] = (rsv.FGMRES, dict(type=rsv.PC_LEARNED, net=net, lnk=lnk32))
        forms.append("fgmres_learned")

    hbm_peak = [0]   # device memory in use (all allocations, torch and the library) after each solve

    def step(profile_headline=False):
        out = {}
        torch.cuda.synchronize()
        ta = time.perf_counter()
        A.update(Bd)
        torch.cuda.synchronize()
        out["assemble_s"] = time.perf_counter() - ta
        for name in forms:
            method, pkw = forms_all[name]
            prof = profile_headline and (name == forms[0] or name == "bicgstab_bilu0")
            t1 = time.perf_counter()
            M = rsv.Precond(A, **pkw)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            x = torch.zeros_like(b)
            if prof:
                # two events per recorded launch: only the classes the roofline needs
                ctx.profile(True, classes=("spmv", "ilu_fwd", "ilu_bwd"))
            st = rsv.solve(A, M, b, x, method=method, restart=30, tol=1e-8, maxit=10000,
                           ortho=(rsv.DCGS2 if name.endswith("_dcgs2") else rsv.CGS2))
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if prof:
                out["kernels_" + name] = ctx.profile_read()
                ctx.profile(False)
            free_b, total_b = torch.cuda.mem_get_info()
            hbm_peak[0] = max(hbm_peak[0], total_b - free_b)
            err = float(torch.linalg.norm(x - xtd) / torch.linalg.norm(xtd))
            out[name] = {"setup_s": t2 - t1, "solve_s": t3 - t2, "its": st["its"], "relres": st["final_relres"],
                         "status": st["status"], "err_vs_xtrue": err, "fallbacks": st["fallbacks"]}
            M.close()
            assert st["status"] == rsv.OK and st["final_relres"] <= 1e-8, (name, st)
        return out

    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: " + ", ".join(f"{k} {r[k]['solve_s'] * 1e3:.1f}ms/{r[k]['its']}its" for k in forms))
    torch.cuda.synchronize()
    res = []
    tt = time.perf_counter()
    for s in range(args.steps):
        r = step(profile_headline=True)
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
    # live kernel timing (HIP events on the solver stream), per profiled form
    ab_global = algorithmic_bytes(cfg.nx, cfg.ny, cfg.nz)
    ab_ras = None

    def kernel_table(form):
        nonlocal ab_ras
        kms = {k: sum(r["kernels_" + form][k][0] for r in res) for k in rsv.K_NAMES}
        kcnt = {k: sum(r["kernels_" + form][k][1] for r in res) for k in rsv.K_NAMES}
        ab = dict(ab_global)
        if forms_all[form][0] != rsv.BICGSTAB:
            # GMRES products (y = A z with ||y||^2) read no third vector; the few
            # residual launches per solve that do read b are counted the same
            ab["spmv"] = ab_global["spmv_plain"]
        if forms_all[form][1].get("type") == rsv.PC_RAS:
            # the sweeps of this form are the local RAS sweeps
            pk = forms_all[form][1]
            ab_ras = ras_algorithmic_bytes(cfg.nx, cfg.ny, cfg.nz, (pk["ras_px"], pk["ras_py"], pk["ras_pz"]),
                                           pk["ras_overlap"])
            ab["ilu_fwd"], ab["ilu_bwd"] = ab_ras["ilu_fwd"], ab_ras["ilu_bwd"]
        tab = {k: {"avg_us": 1e3 * kms[k] / kcnt[k], "launches": kcnt[k],
                   "GBps": (ab[k] / (kms[k] / kcnt[k] * 1e-3) / 1e9) if k in ab and k != "ilu_apply" else None}
               for k in rsv.K_NAMES if kcnt[k] > 0}
        return kms, kcnt, ab, tab

    kms, kcnt, ab, kernels_head = kernel_table(head)
    cand = [k for k in ("spmv", "ilu_fwd", "ilu_bwd") if kcnt[k] > 0]
    dom = max(cand, key=lambda k: kms[k])
    avg_ms = kms[dom] / kcnt[dom]
    achieved = ab[dom] / (avg_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tj = json.load(open(tpath))
            if tj.get("workload") == args.workload:
                traffic = tj["forms"][head]["kernels"][dom]["bytes_per_launch"]
        except Exception:  # noqa: BLE001
            traffic = None
    roofline = {"bound": "hbm", "kernel": dom, "form": head, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": ab[dom], "avg_launch_us": round(avg_ms * 1e3, 2)}
    # the global BILU0 and SpMV kernels, from the BiCGSTAB + BILU0 solves
    kernels = None
    ilu_GBps = spmv_GBps = None
    if "bicgstab_bilu0" in forms:
        bk_ms, bk_cnt, bab, kernels = kernel_table("bicgstab_bilu0")
        if bk_cnt["ilu_fwd"]:
            ilu_ms = (bk_ms["ilu_fwd"] + bk_ms["ilu_bwd"]) / bk_cnt["ilu_fwd"]
            ilu_GBps = round(bab["ilu_apply"] / (ilu_ms * 1e-3) / 1e9, 1)
        spmv_GBps = kernels.get("spmv", {}).get("GBps")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        t0 = time.perf_counter()
        Ao = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, B)
        bo = Ao.spmv(xt)
        t1 = time.perf_counter()
        method, pk = forms_all[head]
        if pk.get("type") == rsv.PC_RAS:
            F = O.RAS(Ao, (cfg.nx, cfg.ny, cfg.nz), (pk["ras_px"], pk["ras_py"], pk["ras_pz"]), pk["ras_overlap"])
            ro = O.gmres(Ao, bo, pc=F, m=30, tol=1e-8, maxit=10000)
            what = "GMRES(30)+RAS(%dx%dx%d, overlap %d) solve (RAS setup" % (pk["ras_px"], pk["ras_py"], pk["ras_pz"],
                                                                          pk["ras_overlap"])
        else:
            F = O.ILU(Ao)
            ro = O.bicgstab(Ao, bo, pc=F, tol=1e-8, maxit=10000)
            what = "BiCGSTAB+BILU0 solve (ILU(0) setup"
        t2 = time.perf_counter()
        cpu = {"value": round(t2 - t1, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"full {args.workload} {what} + {ro['its']} iterations, "
                         f"relres {ro['relres']:.2e}), serial FP64 C on one host thread "
                         f"(the host has {os.cpu_count()} logical cores)"}
        log(f"oracle: {t2 - t1:.2f}s ({ro['its']} its)")

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
    roofline["d2d_copy_GBps"] = copy_GBps

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
        "config": {"workload": f"{args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz} 3x3-block 7-point, "
                               f"headline {head}, tol 1e-8", "unknowns": 3 * cfg.ncell,
                   "forms": forms, "seed": args.seed},
        "solves": summary,
        "vs_plain_gmres_bilu0": ({f: round(summary[f]["solve_s"] / summary["gmres_bilu0"]["solve_s"], 3) for f in forms}
                                 if "gmres_bilu0" in summary else None),
        "learned_training": training,
        # unknowns x iterations per second of the headline solve, beside the paper's
        # closest published figure (scalar Poisson on a CPU cluster): context only
        "unknown_iterations_per_s": round(3 * cfg.ncell * summary[head]["its"] / value, 1),
        "paper_context": {"workload": "scalar 7-point Poisson, 3e9 unknowns, GMRES(30) + RAS(overlap 1, ILU(0)), "
                                      "90 iterations (Poisson Equation example)",
                          "hardware": "IBM Blue Gene/Q, 512 cores (PowerPC A2)",
                          "solve_s": 606.33, "unknown_iterations_per_s": round(3e9 * 90 / 606.33, 1),
                          "note": "solve time = overall - gridding - building - assemble of its 512-core row"},
        "ilu_apply_GBps": ilu_GBps,
        "spmv_GBps": spmv_GBps,
        "kernels": kernels,
        "kernels_headline": kernels_head,
        "ras_local": ab_ras,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "assemble_from_host_s": round(host_assemble_s, 4),
        "assemble_from_host_GBps": round(B.nbytes / host_assemble_s / 1e9, 2),
        "device_bytes": A.device_bytes,
        "hbm_used_bytes": int(hbm_peak[0]),
        "hbm_total_bytes": int(torch.cuda.mem_get_info()[1]),
        "device": ctx.device_info(),
    }
    print(json.dumps(line), flush=True)
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1073741824 bytes read, 1073741824 bytes written")
    A.close(); g.close(); ctx.close()


if __name__ == "__main__":
    main()
