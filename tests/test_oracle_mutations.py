"""The pins catch plausible mistakes: each case plants one mistake in a copy
of the oracle's C source (on the CPU), builds it, and runs the pin that
should catch it against the mutated build, which must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vesis_oracle.c")

# (name, text to replace, replacement, pin test that must fail)
MUTATIONS = [
    ("lj_sign", "lj += 4.0 * s->eps[i] * (sr6 * sr6 - sr6);",
     "lj += 4.0 * s->eps[i] * (sr6 * sr6 + sr6);", "test_lj_sphere_energy_closed_form"),
    ("lj_no_rho", "*u_lj = s->rho_w * lj;", "*u_lj = lj;", "test_lj_sphere_energy_closed_form"),
    ("cfa_no_cross_terms", "ex += f * dx;", "ex += fabs(f * dx);",
     "test_two_charge_cfa_exterior_of_ball_closed_form"),
    ("cfa_prefactor", "return s->coulomb_k / (8.0 * M_PI)", "return s->coulomb_k / (4.0 * M_PI)",
     "test_born_energy_closed_form"),
    ("far_jacobian", "* wt * L / (tau * tau * tau * tau);", "* wt * L / (tau * tau * tau);",
     "test_far_field_centred_atom_independent_integral"),
    ("far_face_axis", "y[a1] = L * gx[iu];", "y[a1] = L * gx[iv];",
     "test_far_field_off_centre_atom_independent_integral"),
    ("surface_power", "pow(s->h, 6) / pow(delta, 4)", "pow(s->h, 4) / pow(delta, 4)",
     "test_geom_energy_of_a_cube_matches_pair_count"),
    ("c0_value", "return 8.0 * M_PI / (M_PI * M_PI - 3.0);", "return 8.0 * M_PI / (M_PI * M_PI - 2.0);",
     "test_C0_matches_its_defining_integral"),
    ("delta_e_sign", "return pref * sum_w - pref * sum_m - h3 * u[j];",
     "return pref * sum_w - pref * sum_m + h3 * u[j];",
     "test_delta_e_equals_energy_difference_of_a_flip"),
    ("band_index", "label_at(s, phi, i, jj - 1, k) != me", "label_at(s, phi, i, jj - 2, k) != me",
     "test_band_is_face_neighbour_disagreement"),
    ("outside_is_solute", "if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 1;",
     "if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return -1;",
     "test_band_is_face_neighbour_disagreement"),
    ("cell_centre_offset", "x[1] = s->center[1] - L + ((double)j + 0.5) * s->h;",
     "x[1] = s->center[1] - L + ((double)j + 0.25) * s->h;",
     "test_cube_symmetry_invariance_of_energy_and_forces"),
    ("colour_period", "int p = (int)ceil(s->rho_s);\n    int64_t cap",
     "int p = (int)ceil(s->rho_s) - 1;\n    int64_t cap",
     "test_colour_pass_energy_change_is_sum_of_flip_changes"),
    ("force_drops_dd_term", "double gx = -qn * (e[0] / r3 - 3.0 * ed * dx / r5);",
     "double gx = -qn * (e[0] / r3);", "test_forces_match_central_differences"),
    ("force_lj_factor", "double clj = s->rho_w * 24.0 * s->eps[nidx]",
     "double clj = s->rho_w * 12.0 * s->eps[nidx]", "test_forces_match_central_differences"),
    ("mobility_grows", "st->M *= st->alpha;", "st->M /= st->alpha;",
     "test_adaptive_mobility_shrinks_after_an_overshoot"),
    ("tight_radius_sign", "double v = sqrt(dx * dx + dy * dy + dz * dz) - d[i];",
     "double v = sqrt(dx * dx + dy * dy + dz * dz) + d[i];",
     "test_tight_start_of_centred_atom_is_the_loose_sphere"),
    ("heap_keeps_stale_entries", "                    ++ver[c];\n", "",
     "test_heap_and_colour_schedules_agree_on_single_atom"),
    ("relax_skips_interface",
     "        orc_minimize_colour(&s, phi, u, o->max_sweeps, 0.0, stats, NULL, NULL, 0);\n", "",
     "test_paper_two_atom_relaxation_reaches_printed_state"),
    ("bend_half_missing", "e += 0.5 * t->kang[a] * (th - t->theta0[a])",
     "e += t->kang[a] * (th - t->theta0[a])", "test_oracle_solute.py::test_bend_energy_closed_form"),
    ("bend_grad_k_as_printed",
     "double gk = pre * (c * qjk[d] / (ljk * ljk) - qji[d] / (lji * ljk));",
     "double gk = pre * (c * qji[d] / (ljk * ljk) - qji[d] / (lji * ljk));",
     "test_oracle_solute.py::test_ss_forces_match_central_differences"),
    ("torsion_plane_orientation", "    cross3(q2, q3, v);\n    double c = dot3(u, v)",
     "    cross3(q3, q2, v);\n    double c = dot3(u, v)",
     "test_oracle_solute.py::test_torsion_energy_closed_form"),
    ("torsion_poly_sign", "double dW = (cp[1] - 3.0 * cp[3] + 5.0 * cp[5])",
     "double dW = (cp[1] + 3.0 * cp[3] + 5.0 * cp[5])",
     "test_oracle_solute.py::test_ss_forces_match_central_differences"),
    ("torsion_grad_j_sign", "g[3 * id[1] + d] += dW * (g1 - g2);",
     "g[3 * id[1] + d] += dW * (g2 - g1);",
     "test_oracle_solute.py::test_ss_forces_are_internal"),
    ("lj_mixing_geometric", "double sg = 0.5 * (t->sigma_ss[i] + t->sigma_ss[j]);",
     "double sg = sqrt(t->sigma_ss[i] * t->sigma_ss[j]);",
     "test_oracle_solute.py::test_nonbonded_pair_closed_forms"),
    ("coulomb_solute_permittivity",
     "double kq = s->coulomb_k * s->q[i] * s->q[j] / s->eps_w;",
     "double kq = s->coulomb_k * s->q[i] * s->q[j] / s->eps_m;",
     "test_oracle_solute.py::test_nonbonded_pair_closed_forms"),
    ("exclusions_ignored", "            if (excluded(keys, t->nexcl, na, i, j)) continue;\n", "",
     "test_oracle_solute.py::test_exclusions_remove_exactly_the_listed_pairs"),
    ("pair_force_drops_coulomb", "*du = (4.0 * ep * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r - kq / r2) / r;",
     "*du = (4.0 * ep * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r) / r;",
     "test_oracle_solute.py::test_ss_forces_match_central_differences"),
    ("subset_drops_far_field",
     "            gx += fw[p] * g[0];\n            gy += fw[p] * g[1];\n"
     "            gz += fw[p] * g[2];\n", "",
     "test_forces_subset_equals_the_rows_of_the_full_forces"),
    ("subset_bond_sign_on_j", "(r - r0[b]) / r * (i == a ? 1.0 : -1.0);",
     "(r - r0[b]) / r * (i == a ? 1.0 : 1.0);",
     "test_forces_subset_equals_the_rows_of_the_full_forces"),
    ("total_forces_skip_solute","        for (int64_t k = 0; k < 3 * s->na; ++k) f[k] -= g[k];\n", "",
     "test_oracle_solute.py::test_total_forces_include_the_solute_terms"),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(name, old, new, pin, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation {name}: pattern must occur exactly once"
    mutated = tmp_path / "vesis_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build(src=str(mutated), lib=str(tmp_path / "liboracle_mut.so"))
    env = dict(os.environ, VESIS_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        f"tests/{pin}" if "::" in pin else f"tests/test_oracle_pins.py::{pin}"],
                       cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"{pin} did not catch {name}:\n{r.stdout[-2000:]}"
