"""The pins must catch plausible mistakes: each mutant below is the oracle's
C source with one planted error, compiled on the CPU; the oracle pin suite
must fail against every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "octaoctree_oracle.c")

MUTANTS = {
    "fold_sequential": ("double fy = (1.0 - fabs(ux)) * sign_pos(uy);",
                        "double fy = (1.0 - fabs(fx)) * sign_pos(uy);"),
    "seam_no_mirror": ("      i = -1 - i;\n      j = R - 1 - j;", "      i = -1 - i;"),
    "tap_weight_swapped": ("w[k] = (a ? fu : 1.0 - fu) * (bb ? fv : 1.0 - fv);",
                           "w[k] = (a ? 1.0 - fu : fu) * (bb ? fv : 1.0 - fv);"),
    "octant_axes_swapped": ("return bx | (by << 1) | (bz << 2);", "return bz | (by << 1) | (bx << 2);"),
    "descent_popcount_off_by_one": ("cur = first + popcount8(mask & ((1u << o) - 1u));",
                                    "cur = first + popcount8(mask & ((2u << o) - 1u));"),
    "refine_at_threshold": ("if (cnt <= tau) continue; /* leaf */", "if (cnt < tau) continue; /* leaf */"),
    "bias_dropped": ("double z = (double)m->b[i][o];", "double z = 0.0;"),
    "ggx_denominator_unsquared": ("double Dm = a2 / (PI * den * den);", "double Dm = a2 / (PI * den);"),
    "fresnel_wrong_power": ("pow(1.0 - dot3(wi, hv), 5.0)", "pow(1.0 - dot3(wi, hv), 4.0)"),
    "rhs_mean_missing": ("T[3 * b + c] += acc / (double)N;", "T[3 * b + c] += acc;"),
    "residual_sign": ("r[i] = lhs[i] - T[i];", "r[i] = T[i] - lhs[i];"),
    "loss_mean_over_B": ("*loss_out = B > 0 ? acc / (3.0 * (double)B) : 0.0;",
                         "*loss_out = B > 0 ? acc / (double)B : 0.0;"),
    "backprop_transposed_weight": ("s += (double)m->W[i][(int64_t)o * fin + k] * delta[o];",
                                   "s += (double)m->W[i][(int64_t)k * fout + o] * delta[o];"),
    "relu_mask_missing": ("if (i > 0 && !(pre[i - 1][k] > 0.0)) s = 0.0;", ""),
    "scatter_wrong_tap_weight": ("dfeat[l][base + c] += qt->w[l][k] * dh[l * C + c];",
                                 "dfeat[l][base + c] += 0.25 * dh[l * C + c];"),
    "node_offset_dropped": ("int64_t local = (int64_t)idx - t->level_offset[l];\n  return ((local * R + j) * R + i) * t->C;",
                            "int64_t local = 0;\n  return ((local * R + j) * R + i) * t->C;"),
    # the paper's interpolation (Sec. 3.3 vertex maps, Sec. 3.4 8-cell blend)
    "paper_node_offset_dropped": ("int64_t local = (int64_t)idx - t->level_offset[l];\n  return (local * ora_map_entries",
                                  "int64_t local = 0;\n  return (local * ora_map_entries"),
    "bary_diagonal_flipped": ("int same_side = (2 * i >= R) == (2 * j >= R);",
                              "int same_side = (2 * i >= R) != (2 * j >= R);"),
    "bary_weight_swapped": ("v[1][0] = i + 1; v[1][1] = j;     w[1] = fu;", "v[1][0] = i + 1; v[1][1] = j;     w[1] = fv;"),
    "vertex_seam_not_shared": ("  if (i == 0 || i == R) j = j < R - j ? j : R - j;\n", ""),
    "trilinear_not_renormalised": ("for (int d = 0; d < 8; ++d) w[d] = sum > 0.0 ? w[d] / sum : 0.0;", ""),
    "trilinear_centre_offset_dropped": ("double p = xa * ldexp(1.0, l) - 0.5;", "double p = xa * ldexp(1.0, l);"),
    "paper_scatter_wrong_weight": ("          for (int32_t c = 0; c < C; ++c) dfeat[l][base + c] += wk * dh[l * C + c];",
                                   "          for (int32_t c = 0; c < C; ++c) dfeat[l][base + c] += qt->vw[l][d][k] * dh[l * C + c];"),
    # the optimiser step
    "adam_no_bias_correction": ("double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);",
                                "double c1 = 1.0, c2 = 1.0 - pow(b2, (double)t);"),
    "adam_untouched_updated": ("    if (touched && !touched[i / block]) continue;\n", ""),
    "adam_second_moment_unsquared": ("double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;",
                                     "double vi = b2 * (double)v[i] + (1.0 - b2) * fabs(gi);"),
    # the decoder's surface attributes (Sec. 3.5)
    "attribute_order_reversed": ("for (int32_t k = 0; k < E; ++k) h[LC + k] = (double)e[k];",
                                 "for (int32_t k = 0; k < E; ++k) h[LC + E - 1 - k] = (double)e[k];"),
    "rhs_backward_reads_lhs_attributes": ("*e = E > 0 ? &bt->attr2[E * bk] : NULL;",
                                          "*e = E > 0 ? &bt->attr[E * b] : NULL;"),
    "backward_reads_first_point_attributes": ("*e = E > 0 ? &bt->attr[E * q] : NULL;",
                                              "*e = E > 0 ? &bt->attr[0] : NULL;"),
    # the disparity-shifted lookup (Sec. 3.3) and its predictor (Sec. 3.5)
    "shift_centre_offset_dropped": ("dv[a] = xc[a] - ((double)cells[3 * d + a] + 0.5) / ldexp(1.0, l);",
                                    "dv[a] = xc[a] - ((double)cells[3 * d + a]) / ldexp(1.0, l);"),
    "shift_sign_flipped": ("v[a] = dv[a] * qt->disp + u[a];", "v[a] = -dv[a] * qt->disp + u[a];"),
    "shift_direction_not_unit": ("    unit_dir(d3, u);\n    for (int a = 0; a < 3; ++a) {\n      double xa",
                                 "    for (int a = 0; a < 3; ++a) u[a] = d3[a];\n    for (int a = 0; a < 3; ++a) {\n"
                                 "      double xa"),
    "octa_jacobian_fold_sign": ("double fx = -sx * sy * du[1][b], fy = -sx * sy * du[0][b];",
                                "double fx = sx * sy * du[1][b], fy = sx * sy * du[0][b];"),
    "bary_derivative_axes_swapped": ("qt->dvw[l][d][k] = R * (gu[k] * ds + gv[k] * dt);",
                                     "qt->dvw[l][d][k] = R * (gu[k] * dt + gv[k] * ds);"),
    "hash_primes_swapped": ("((uint32_t)c[1] * 2654435761u) ^ ((uint32_t)c[2] * 805459861u)",
                            "((uint32_t)c[1] * 805459861u) ^ ((uint32_t)c[2] * 2654435761u)"),
    "hash_dense_stride_dropped": ("return c[0] + N1 * (c[1] + N1 * c[2]);", "return c[0] + N1 * (c[1] + c[2]);"),
    "hash_weight_swapped": ("        wd *= bit ? f[a] : 1.0 - f[a];\n      }\n      int64_t slot = hash_slot",
                            "        wd *= bit ? 1.0 - f[a] : f[a];\n      }\n      int64_t slot = hash_slot"),
    "disparity_gradient_without_cell_weight": ("dd += qt->nbw[l][d] * qt->dvw[l][d][k] * s;",
                                               "dd += qt->dvw[l][d][k] * s;"),
    "hash_scatter_without_vertex_weight": ("+= qt->hw[i][d] * qt->denc[i * g->F + e];",
                                           "+= qt->denc[i * g->F + e];"),
    "predictor_direction_not_unit": ("  unit_dir(d3, u);\n  in[E] = u[0];", "  for (int a = 0; a < 3; ++a) u[a] = d3[a];\n  in[E] = u[0];"),
    "scatter_into_first_node": ("int64_t base = texel_base(t, l, qt->idx[l], qt->ij[l][2 * k], qt->ij[l][2 * k + 1]);\n"
                                "      for (int32_t c = 0; c < C; ++c) dfeat",
                                "int64_t base = texel_base(t, l, (int32_t)t->level_offset[l], qt->ij[l][2 * k], "
                                "qt->ij[l][2 * k + 1]);\n      for (int32_t c = 0; c < C; ++c) dfeat"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    msrc = tmp_path / "octaoctree_oracle.c"
    msrc.write_text(src.replace(old, new))
    (tmp_path / "octaoctree_oracle.h").write_text(open(SRC.replace(".c", ".h")).read())
    lib = tmp_path / "liboo_mutant.so"
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(lib),
                    str(msrc), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    pins = [os.path.join(ROOT, "tests", f) for f in sorted(os.listdir(os.path.join(ROOT, "tests")))
            if f.startswith("test_oracle_") and f != "test_oracle_mutants.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "--hypothesis-seed=0"] + pins, env=env, capture_output=True, text=True, timeout=600,
                       cwd=ROOT)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
