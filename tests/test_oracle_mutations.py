"""The pins have teeth: plant one plausible mistake at a time in a copy of
the oracle's C source (on the CPU), build it, and check that some pin fails.

(Ranging the evader's switching function over the whole costate box instead
of the half the pursuer's branch leaves is an equivalent mutant for the
pursuit-evasion game: any input pair it adds is matched by a realised pair
with the same |f_d|, so no pin can see it; it is not listed.)

Each mutant is a single textual change to oracle/odp_oracle.c; the test
first asserts the original text is present, so a refactor of the oracle that
moves a site makes this test fail loudly instead of silently passing.
"""
import os
import subprocess

import numpy as np
import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "odp_oracle.c")

MUTANTS = [
    ("lf_sign", "diss += 0.5 * alpha[d] * (pp[d] - pm[d]);",
     "diss -= 0.5 * alpha[d] * (pp[d] - pm[d]);"),
    ("lf_dropped_on_last_axis", "for (int d = 0; d < N; ++d) diss += 0.5",
     "for (int d = 0; d < N - 1; ++d) diss += 0.5"),
    ("one_sided_swapped", "double dm = wc - wl, dp = wr - wc;", "double dm = wr - wc, dp = wc - wl;"),
    ("costate_not_halved", "pbar[d] = 0.5 * (pp[d] + pm[d]);", "pbar[d] = (pp[d] + pm[d]);"),
    ("ghost_toward_zero", "return vb + (double)m * og_sgn(vb) * fabs(vb - vin);",
     "return vb - (double)m * og_sgn(vb) * fabs(vb - vin);"),
    ("second_ghost_like_first", "return vb + (double)m * og_sgn(vb) * fabs(vb - vin);",
     "return vb + og_sgn(vb) * fabs(vb - vin);"),
    ("eno_choice_inverted", "return fabs(x) <= fabs(y);", "return fabs(x) > fabs(y);"),
    ("eno_correction_sign", "dm = dm + 0.5 * (fm ? sm : s0);", "dm = dm - 0.5 * (fm ? sm : s0);"),
    ("eno_plus_side_stencils_shifted", "int fp = eno_f32 ? og_eno_first_f32(wl, wc, wr, wrr) : og_eno_first(s0, sp);\n            dm = dm + 0.5 * (fm ? sm : s0);\n            dp = dp - 0.5 * (fp ? s0 : sp);",
     "int fp = eno_f32 ? og_eno_first_f32(wl, wc, wr, wrr) : og_eno_first(s0, sp);\n            dm = dm + 0.5 * (fm ? sm : s0);\n            dp = dp - 0.5 * (fp ? sm : s0);"),
    ("eno_correction_not_halved", "dp = dp - 0.5 * (fp ? s0 : sp);", "dp = dp - (fp ? s0 : sp);"),
    ("periodic_wrap_off_by_one", "long kw = (k + g->n[d]) % g->n[d];",
     "long kw = (k + g->n[d] + 1) % g->n[d];"),
    ("cos_sin_swapped_3d", "f[0] = dy->p[0] * cos(z[2]);\n        f[1] = dy->p[0] * sin(z[2]);\n        f[2] = u[0];\n        break;\n    case OG_DYNCAR4D",
     "f[0] = dy->p[0] * sin(z[2]);\n        f[1] = dy->p[0] * cos(z[2]);\n        f[2] = u[0];\n        break;\n    case OG_DYNCAR4D"),
    ("pursuer_uses_evader_heading", "f[3] = dy->p[2] * cos(z[5]);", "f[3] = dy->p[2] * cos(z[2]);"),
    ("car_speed_axis_wrong", "f[0] = z[2] * cos(z[3]);", "f[0] = z[3] * cos(z[3]);"),
    ("bang_bang_inverted", "if (maximise) return s >= 0.0 ? bound : -bound;",
     "if (maximise) return s >= 0.0 ? -bound : bound;"),
    ("ball_input_sign", "double sgn = dy->u_mode ? 1.0 : -1.0;",
     "double sgn = dy->u_mode ? -1.0 : 1.0;"),
    ("drift_sign", "f[d] = dy->p[1 + d] + u[d];", "f[d] = -dy->p[1 + d] + u[d];"),
    ("rk3_weight", "if (order == 3 && stage == 1) { *a = 0.75; *b = 0.25; }",
     "if (order == 3 && stage == 1) { *a = 0.5; *b = 0.5; }"),
    ("rk2_weight", "if (order == 2 && stage == 1) { *a = 0.5; *b = 0.5; }",
     "if (order == 2 && stage == 1) { *a = 0.0; *b = 1.0; }"),
    ("cfl_number_dropped", "double dt = cfl / s;", "double dt = 1.0 / s;"),
    ("tube_clamp_max", "if (ref < v) v = ref;", "if (ref > v) v = ref;"),
    ("value_over_time_uses_v0", "(tmode <= 4) ? Vn[i] : target[i];", "(tmode <= 4) ? V0[i] : target[i];"),
    ("target_uses_v0", "(tmode <= 4) ? Vn[i] : target[i];", "(tmode <= 4) ? Vn[i] : V0[i];"),
    ("obstacle_max_as_min", "if (omode == 2 && obstacle[i] > v) v = obstacle[i];",
     "if (omode == 2 && obstacle[i] < v) v = obstacle[i];"),
    ("max_methods_as_min", "if (tmode % 2 == 1) {", "if (tmode % 2 == 0 || tmode == 1) {"),
    ("set_slice_off_by_one", "const size_t off = set_slices > 1 ? (size_t)(k - 1) * (size_t)P : 0;",
     "const size_t off = set_slices > 1 ? (size_t)k * (size_t)P : 0;"),
    ("set_slices_ignored", "const size_t off = set_slices > 1 ? (size_t)(k - 1) * (size_t)P : 0;",
     "const size_t off = 0;"),
    ("pe3d_switching_mixed_sign", "u[0] = og_bang(pbar[0] * z[1] - pbar[1] * z[0] - pbar[2],",
     "u[0] = og_bang(pbar[0] * z[1] + pbar[1] * z[0] - pbar[2],"),
    ("pe3d_ydot_cos", "f[1] = dy->p[1] * sin(z[2]) - u[0] * z[0];", "f[1] = dy->p[1] * cos(z[2]) - u[0] * z[0];"),
    ("pe3d_heading_rate_sign", "f[2] = dd[0] - u[0];", "f[2] = u[0] - dd[0];"),
    ("pe3d_speeds_exchanged", "f[0] = -dy->p[0] + dy->p[1] * cos(z[2]) + u[0] * z[1];",
     "f[0] = -dy->p[1] + dy->p[0] * cos(z[2]) + u[0] * z[1];"),
    ("pe3d_cfl_from_all_inputs", "og_alpha_box_max(&g, &dy, box0, amax);", "og_alpha_max(&g, &dy, amax);"),
    ("global_alpha_ignored", "const double *aglob = global_alpha ? amax : NULL;", "const double *aglob = NULL;"),
    ("global_alpha_axis0_for_all", "for (int d = 0; d < N; ++d) alpha[d] = alpha_glob[d];",
     "for (int d = 0; d < N; ++d) alpha[d] = alpha_glob[0];"),
    ("eno_f32_tie_to_second", "    return fabsf(x) <= fabsf(y);", "    return fabsf(x) < fabsf(y);"),
    ("eno_f32_decides_in_float64", "    return fabsf(x) <= fabsf(y);",
     "    return fabs((w2 - w1) - (w1 - w0)) <= fabs((w3 - w2) - (w2 - w1));"),
    ("ttr_jacobi_reads_new_iterate", "og_field F = {og_get_array, jacobi ? old : phi, NULL, 0};",
     "og_field F = {og_get_array, phi, NULL, 0};"),
    ("ttr_jacobi_edge_reads_new_iterate", "const double *src = jacobi ? old : phi;", "const double *src = phi;"),
    ("costate_box_not_used", "static int og_box_dynamics(const og_dyn *dy) { return dy->id == OG_PE3D; }",
     "static int og_box_dynamics(const og_dyn *dy) { return dy->id < 0; }"),
    ("ttr_right_side_dropped", "double H = 0.0, num = 1.0, den = 0.0;", "double H = 0.0, num = 0.0, den = 0.0;"),
    ("ttr_hamiltonian_sign", "num += H;", "num -= H;"),
    ("ttr_sigma_not_used_in_sum", "num += sig[d] * nsum[d] / (2.0 * g.dx[d]);", "num += nsum[d] / (2.0 * g.dx[d]);"),
    ("last_step_not_clipped", "dt = tau[k] - t;", "dt = dt + 0.0;"),
    ("control_bound_for_disturbance", "dd[0] = og_bang(pbar[5], dy->p[3], dy->d_mode);",
     "dd[0] = og_bang(pbar[5], dy->p[1], dy->d_mode);"),
    ("car_controls_exchanged", "u[0] = og_bang(pbar[2], dy->p[0], dy->u_mode);\n        u[1] = og_bang(pbar[3], dy->p[1], dy->u_mode);",
     "u[0] = og_bang(pbar[2], dy->p[1], dy->u_mode);\n        u[1] = og_bang(pbar[3], dy->p[0], dy->u_mode);"),
    ("periodic_spacing_like_closed", "g->dx[d] = g->periodic[d] ? (hi[d] - lo[d]) / (double)n[d]",
     "g->dx[d] = g->periodic[d] ? (hi[d] - lo[d]) / (double)(n[d] - 1)"),
]

FAST_PINS = [
    lambda o: [pins.test_pin1_hopf_lax(o, *c) for c in pins.CASES_PIN1],
    lambda o: [pins.test_pin1b_bang_bang_axis_closed_form(o, *c) for c in pins.ONE_AXIS],
    lambda o: pins.test_pin2_periodic_shift_at_cfl_one(o),
    lambda o: [pins.test_pin2_upwind_identity(o, c, f) for c, f in [(0.8, 0.5), (-1.3, 0.9)]],
    lambda o: pins.test_pin2_dubins_x_axis_slice(o),
    lambda o: [pins.test_pin3_brt_monotone(o, w, r) for w, r in [("dubins3d", 1), ("dyncar4d", 3)]],
    lambda o: pins.test_pin4_dubins_symmetries(o),
    lambda o: pins.test_pin4_car_and_game_mirror(o),
    lambda o: [pins.test_pin5_game_separates(o, p) for p in ("evader", "pursuer")],
    lambda o: pins.test_pin6_car_reduces_to_dubins(o),
    lambda o: [pins.test_pin8_rk_temporal_order(o, r) for r in (1, 2, 3)],
    lambda o: pins.test_golden_step_count_3d(o),
    lambda o: pins.test_restart_equals_single_call(o),
    lambda o: [pins.test_pin9_computation_methods_closed_form(o, *c, f) for c in pins.CASES_PIN9
               for f in (1.0, 0.5)],
    lambda o: [pins.test_pin9_time_varying_sets(o, f) for f in (1.0, 0.5)],
    lambda o: [pins.test_pin10_eno2_exact_on_quadratics(o, n) for n in (1, 3)],
    pins.test_pin10_eno2_picks_the_smooth_side,
    pins.test_pin10_eno2_tie_takes_the_first_stencil,
    pins.test_pin10_eno2_second_ghost,
    pins.test_pin11_pe3d_hamiltonian_is_max_min,
    pins.test_pin11_alpha_box_brute_force,
    pins.test_pin11_pe3d_without_turning_is_drift,
    pins.test_pin11_pe3d_one_step_with_known_box,
    pins.test_pin11_pe3d_cfl_step_from_the_box,
    pins.test_pin11_pe3d_capture_box_is_all_inputs,
    pins.test_pin11_pe3d_mirror_symmetry,
    pins.test_pin12_ttr_ball_closed_form_first_order,
    pins.test_pin12_ttr_speed_scaling,
    pins.test_pin12_ttr_dubins_straight_ahead,
    pins.test_pin13_global_alpha_heat_step_where_the_drift_vanishes,
    pins.test_pin13_global_alpha_converges_at_first_order,
    pins.test_pin13_global_alpha_tube_monotone,
    pins.test_pin14_eno_f32_choices_agree_with_margins,
    pins.test_pin14_eno_f32_near_tie_built_by_hand,
    pins.test_pin15_ttr_jacobi_front_in_1d,
    lambda o: [pins.test_pin9_restart_reference(o, m, f) for m, f in
               (("minVWithVInit", np.minimum), ("maxVWithVInit", np.maximum), ("minVWithV0", None))],
]


def _first_failing_pin(oracle_mod):
    for k, pin in enumerate(FAST_PINS):
        try:
            pin(oracle_mod)
        except (AssertionError, ValueError, FloatingPointError):
            return k
    return None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(oracle_mod, tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} moved"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-o", str(lib), str(mut), "-lm"])
    with oracle_mod.use_library(str(lib)):
        caught = _first_failing_pin(oracle_mod)
    assert caught is not None, f"no pin catches mutant {name}"


def test_unmutated_passes_fast_pins(oracle_mod):
    assert _first_failing_pin(oracle_mod) is None
