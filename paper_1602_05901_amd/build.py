"""Build step for the native parts: the HIP solver library (gfx950), the
seeded input generator and the CPU oracle used by the tests.

    python -m paper_1602_05901_amd.build          # everything
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = [
    "csrc/rsv_core.hip",
    "csrc/rsv_kernels.hip",
    "csrc/rsv_ilu.hip",
    "csrc/rsv_ras.hip",
    "csrc/rsv_krylov.hip",
    "csrc/rsv_unet.hip",
    "csrc/rsv_hsfc.hip",
    "csrc/rsv_scalar.hip",
    "csrc/rsv_iluk.hip",
    "csrc/rsv_cpr.hip",
]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def _run(cmd, cwd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, cwd=cwd, check=True)


def build_gen():
    d = os.path.join(PKG, "inputs")
    _run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", "libgen.so", "gen.c", "-lm"], d)


def build_oracle():
    d = os.path.join(ROOT, "oracle")
    srcs = [s for s in ("oracle.c", "unet.c", "hsfc.c", "scalar.c", "mg.c", "cpr.c", "ilut.c") if os.path.exists(os.path.join(d, s))]
    _run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", "liboracle.so", *srcs, "-lm"], d)


def build_hip():
    srcs = [s for s in HIP_SOURCES if os.path.exists(os.path.join(PKG, s))]
    out = os.path.join(PKG, "librsv.so")
    tmp = out + ".tmp"
    _run([HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs], PKG)
    os.replace(tmp, out)


def build_all():
    build_gen()
    build_oracle()
    build_hip()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"all": build_all, "gen": build_gen, "oracle": build_oracle, "hip": build_hip}[w]()
