"""CPU-side checks of the C ABI: the library loads, exports every function
that include/rsv.h declares, and the Python structs match the C layout.
No GPU work is issued."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsv.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rsv_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["rsv_create", "rsv_grid_create", "rsv_cell_to_row", "rsv_matrix_assemble", "rsv_spmv",
                 "rsv_precond_setup", "rsv_precond_apply", "rsv_solve", "rsv_net_train_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1602_05901_amd import rsv
    L = rsv.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # exported with C linkage (no mangling)
    out = subprocess.run(["nm", "-D", "--defined-only", rsv.LIB_PATH], capture_output=True, text=True).stdout
    for n in declared_functions():
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_binding_covers_header():
    from paper_1602_05901_amd import rsv
    assert set(declared_functions()) == set(rsv._SIGS)


def test_status_strings_and_version():
    from paper_1602_05901_amd import rsv
    L = rsv.lib()
    assert L.rsv_version() == 10000
    assert L.rsv_status_str(rsv.ERR_ZERO_PIVOT) == b"RSV_ERR_ZERO_PIVOT"
    assert L.rsv_status_str(rsv.NOT_CONVERGED) == b"RSV_NOT_CONVERGED"


def test_struct_layouts_match_c(tmp_path):
    from paper_1602_05901_amd import rsv
    src = tmp_path / "sz.c"
    src.write_text('#include "rsv.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rsv_pc_params), '
                   'sizeof(rsv_solver_params), sizeof(rsv_stats), sizeof(rsv_net_arch), '
                   'offsetof(rsv_pc_params, theta), offsetof(rsv_stats, bad_cell));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(rsv.PcParams), ctypes.sizeof(rsv.SolverParams), ctypes.sizeof(rsv.Stats),
                    ctypes.sizeof(rsv.NetArch), rsv.PcParams.theta.offset, rsv.Stats.bad_cell.offset]


def test_defaults_follow_paper(tmp_path):
    """RAS defaults of the paper's default-parameter figure (overlap 1, ILU level 0)
    and restart 30 of its GMRES(30) runs; read from tests/golden."""
    import json
    from paper_1602_05901_amd import rsv
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_defaults.json")))
    p = rsv.PcParams()
    rsv.lib().rsv_pc_params_default(ctypes.byref(p))
    assert p.ras_overlap == gold["ras"]["overlap"]
    assert p.iluk_level == gold["ras"]["iluk_level"]
    assert p.local_solver == rsv.LOCAL_ILUK                 # the figure's default solver ILUK
    assert p.ilut_p == gold["ras"]["ilut_p"] and p.ilut_tol == gold["ras"]["ilut_tol"]
    s = rsv.SolverParams()
    rsv.lib().rsv_solver_params_default(ctypes.byref(s))
    assert s.restart == gold["gmres_restart"]


def test_no_oracle_in_product_path():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1602_05901_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                txt = open(os.path.join(dp, f), errors="replace").read()
                assert "import oracle" not in txt and "from oracle" not in txt and "oracle.h" not in txt, f
