"""Mutation checks for the oracle's pins: each case plants one plausible slip
in a copy of the oracle's C sources (never in the sources themselves),
builds that copy on the CPU, and runs the pin that should catch it in a
subprocess that loads the broken build (ORACLE_LIB).  The pin must fail;
the unmodified copy built the same way must pass the same pins.  No GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")
PINS = "tests/test_oracle_pins_branches.py"
HP = "tests/test_oracle_hsfc_pins.py"
SP = "tests/test_oracle_scalar_pins.py"
KP = "tests/test_oracle_iluk_pins.py"
CP = "tests/test_oracle_cpr_pins.py"
TP = "tests/test_oracle_ilut_pins.py"

# (id, file, text in the oracle, replacement, pins that must fail)
MUTATIONS = [
    ("adam_bias_exponent", "unet.c", "pow(b1, (double)t)", "b1",
     [PINS + "::test_adam_constant_gradient_steps_2_and_3", PINS + "::test_adam_three_different_gradients_closed_form"]),
    ("adam_second_moment_exponent", "unet.c", "pow(b2, (double)t)", "b2",
     [PINS + "::test_adam_constant_gradient_steps_2_and_3"]),
    ("fgmres_no_cycle_handover", "oracle.c", "if (consecutive_fb >= 3) fb_rest = 1;", "",
     [PINS + "::test_fgmres_three_rejections_hand_the_cycle_to_the_fallback"]),
    ("fgmres_no_reset_on_accept", "oracle.c",
     "if (used_fb) { st->fallbacks++; consecutive_fb++; } else consecutive_fb = 0;",
     "if (used_fb) { st->fallbacks++; consecutive_fb++; }",
     [PINS + "::test_fgmres_acceptance_resets_the_consecutive_count"]),
    ("bicgstab_no_omega_exit", "oracle.c", "if (omega == 0.0) { rc = ORC_BREAKDOWN; break; }", "",
     [PINS + "::test_bicgstab_breakdown_exits[omega0]"]),
    ("hsfc_table_entry", "hsfc.c", "{0, 7, 3, 4, 1, 6, 2, 5},", "{0, 7, 4, 3, 1, 6, 2, 5},",
     [HP + "::test_keys_are_a_bijection_and_consecutive_points_are_neighbours[2]"]),
    ("hsfc_bit_order", "hsfc.c", "const int bit = 31 - l;", "const int bit = 32 - levels + l;",
     [HP + "::test_level_one_order_and_nesting"]),
    ("partition_rank_rounding", "hsfc.c", "part[v[r].idx] = (int32_t)((r * (int64_t)nparts) / n);",
     "part[v[r].idx] = (int32_t)(((r + 1) * (int64_t)nparts - 1) / n);",
     [HP + "::test_partition_is_the_equal_count_cut_of_the_curve"]),
    ("quality_inner_faces_twice", "hsfc.c", "else if (m > c) f[p]++;", "else f[p]++;",
     [HP + "::test_quality_against_brute_force"]),
    ("scalar_ilu_update_sign", "scalar.c", "M->val[where[j]] -= M->val[p] * M->val[q];",
     "M->val[where[j]] += M->val[p] * M->val[q];",
     [SP + "::test_ilu0_characterisation_and_apply"]),
    ("scalar_ras_writes_every_cell", "scalar.c", "if (R->owner[cs[q]] == s) z[cs[q]] = zl[q];", "z[cs[q]] = zl[q];",
     [SP + "::test_ras_on_a_line_is_the_restricted_sum_of_exact_local_solves"]),
    ("iluk_level_sum", "oracle.c", "const int64_t l = lev[m] + levs[q] + 1;", "const int64_t l = lev[m] + levs[q];",
     [KP + "::test_level_one_pattern_of_the_seven_point_stencil[dims0]"]),
    ("iluk_pattern_row_pointer", "oracle.c", "rp[i + 1] = used;   /* row i is read by the rows after it */", "",
     [KP + "::test_level_one_pattern_of_the_seven_point_stencil[dims0]"]),
    ("bicgstab_no_rv_exit", "oracle.c",
     "if (rv == 0.0 || !isfinite(rv)) { rc = isfinite(rv) ? ORC_BREAKDOWN : ORC_ERR_NAN; break; }",
     "if (!isfinite(rv)) { rc = ORC_ERR_NAN; break; }",
     [PINS + "::test_bicgstab_breakdown_exits[rv0]"]),
    ("mg_post_sweep_order", "mg.c",
     "        if ((rc = gs_colour(L, b, x, 1)) != ORC_OK) return rc;\n        if ((rc = gs_colour(L, b, x, 0)) != ORC_OK) return rc;\n    }\n    return ORC_OK;",
     "        if ((rc = gs_colour(L, b, x, 0)) != ORC_OK) return rc;\n        if ((rc = gs_colour(L, b, x, 1)) != ORC_OK) return rc;\n    }\n    return ORC_OK;",
     [CP + "::test_cycle_is_symmetric_for_a_symmetric_matrix"]),
    ("mg_restriction_overwrites", "mg.c", "C->b[aggregate_of(L, i, C->nx, C->ny)] += L->r[i];",
     "C->b[aggregate_of(L, i, C->nx, C->ny)] = L->r[i];",
     [CP + "::test_cycle_error_operator_matches_the_multigrid_recursion"]),
    ("mg_residual_sign", "mg.c", "L->r[i] = b[i] - L->r[i];", "L->r[i] = L->r[i] - b[i];",
     [CP + "::test_cycle_error_operator_matches_the_multigrid_recursion"]),
    ("mg_galerkin_overwrites", "mg.c", "cval[I * MG_ROW_CAP + q] += val[p];", "cval[I * MG_ROW_CAP + q] = val[p];",
     [CP + "::test_levels_are_galerkin_products_on_halved_grids"]),
    ("cpr_fpf_stale_residual", "cpr.c",
     "        residual(P, f, x, P->r);\n        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;\n        break;\n    case ORC_CPR_FFPF:",
     "        if ((rc = smoother_step(P, P->r, x)) != ORC_OK) return rc;\n        break;\n    case ORC_CPR_FFPF:",
     [CP + "::test_error_propagation_is_the_product_of_the_stages"]),
    ("cpr_quasi_impes_sign", "cpr.c", "w[1] = (-d[1] * d[8] + d[7] * d[2]) / det;",
     "w[1] = (d[1] * d[8] - d[7] * d[2]) / det;", [CP + "::test_decoupling_weights"]),
    ("cpr_abf_column_of_the_inverse", "cpr.c", "w[1] = inv[1];\n        w[2] = inv[2];",
     "w[1] = inv[3];\n        w[2] = inv[6];", [CP + "::test_decoupling_weights"]),
    ("cpr_pressure_row_not_column", "cpr.c", "val[p] = w[0] * blk[0] + w[1] * blk[3] + w[2] * blk[6];",
     "val[p] = w[0] * blk[0] + w[1] * blk[1] + w[2] * blk[2];",
     [CP + "::test_pressure_matrix_is_the_restricted_decoupled_matrix"]),
    ("ilut_threshold_not_squared", "ilut.c", "const double thr = (tol * tol) * nrm2;", "const double thr = tol * nrm2;",
     [TP + "::test_first_two_rows_by_hand"]),
    ("ilut_keeps_the_smallest", "ilut.c", "if (vb > va || (vb == va && cand[b] < cand[a])) ++rank;",
     "if (vb < va || (vb == va && cand[b] < cand[a])) ++rank;", [TP + "::test_first_two_rows_by_hand"]),
    ("ilut_update_sign", "ilut.c", "w[9 * j + e] = w[9 * j + e] - prod[e];", "w[9 * j + e] = w[9 * j + e] + prod[e];",
     [TP + "::test_zero_tolerance_is_the_exact_lu"]),
    ("ilut_no_drop_right_of_i", "ilut.c", "if (j > i && present[j] && !(fro2(w + 9 * j) < thr)) cand[m++] = j;",
     "if (j > i && present[j]) cand[m++] = j;", [TP + "::test_kept_blocks_pass_the_drop_test_and_the_count"]),
    ("ilut_l_not_scaled", "ilut.c", "memcpy(w + 9 * k, wk, sizeof(wk));", "",
     [TP + "::test_zero_tolerance_is_the_exact_lu"]),
]


C_SOURCES = ("oracle.c", "unet.c", "hsfc.c", "scalar.c", "mg.c", "cpr.c", "ilut.c")


def _build(tmp, mutation=None):
    src = os.path.join(tmp, "src")
    os.makedirs(src, exist_ok=True)
    for f in C_SOURCES + ("oracle.h",):
        shutil.copy(os.path.join(ORC, f), src)
    if mutation is not None:
        _, fname, old, new, _ = mutation
        path = os.path.join(src, fname)
        text = open(path).read()
        assert text.count(old) == 1, f"mutation site not unique in {fname}: {old!r}"
        open(path, "w").write(text.replace(old, new))
    lib = os.path.join(tmp, "liboracle_mut.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
                    *[os.path.join(src, f) for f in C_SOURCES], "-lm"],
                   check=True)
    return lib


def _run_pins(lib, nodes):
    env = dict(os.environ, ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *nodes],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


def test_unmutated_copy_passes_the_pins(tmp_path):
    lib = _build(str(tmp_path))
    nodes = sorted({n for m in MUTATIONS for n in m[4]})
    r = _run_pins(lib, nodes)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_mutation(tmp_path, mutation):
    lib = _build(str(tmp_path), mutation)
    r = _run_pins(lib, mutation[4])
    # exit code 1: the tests ran and at least one failed (not a crash or a
    # collection error)
    assert r.returncode == 1, r.stdout[-2000:]
    assert "failed" in r.stdout
