"""The pins must be able to fail: each case plants one plausible mistake in a
copy of the oracle's C source (a flipped sign, a dropped term, a wrong index
or upwind side, transposed operands, a wrong breakpoint), builds it, and runs
the oracle pins against it until one fails.  A mistake no pin catches fails
the test.  Everything here runs on the CPU."""
import os
import subprocess

import pytest

import oracle
import test_oracle_constants as T_const
import test_oracle_invariants as T_inv
import test_oracle_noneq as T_noneq
import test_oracle_physics as T_phys
import test_oracle_textbook as T_text

SRC = os.path.join(os.path.dirname(oracle.__file__), "mrtfd_oracle.c")

# the equilibrium ghost state of the x sides (the y sides' line reads the same)
EQX = """/* x-lo, x-hi */
        int kind = p->bc_kind[side];
        const double* st = p->bc_state[side];
        if (kind == ORC_BC_EQUILIBRIUM) feq_velocity(C, p->b, st[0], st[1], st[2], st[3], eq);"""

# the row of M* at the relative velocity of population i
STAR = "if (star) moment_row_values(C.vx[i] - vx, C.vy[i] - vy, C.eta[i], row);"

# the outgoing and incoming limited face values along one axis
FACES = """                    double Fout = fJ + 0.5 * (1.0 - nu) * limited_jump(p->limiter, fJm1, fJ, fJp1);
                    double Fin = fJm1 + 0.5 * (1.0 - nu) * limited_jump(p->limiter, fJm2, fJm1, fJ);"""

# (name, original text, planted mistake)
MUTANTS = [
    ("correction_8_sign", "R[7] += C8;", "R[7] -= C8;"),
    ("correction_9_dropped", "R[8] += C9;", "R[8] += 0.0 * C9;"),
    ("y_upwind_side", "int ex = (a == 0) ? sg : 0, ey = (a == 1) ? sg : 0;",
     "int ex = (a == 0) ? sg : 0, ey = (a == 1) ? -sg : 0;"),
    ("inflow_face_operands", "limited_jump(p->limiter, fJm2, fJm1, fJ);", "limited_jump(p->limiter, fJm1, fJm2, fJ);"),
    ("courant_without_A", "double nu = p->dt / (C->A[i] * ((a == 0) ? p->dx : p->dy));",
     "double nu = p->dt / ((a == 0) ? p->dx : p->dy);"),
    ("temperature_factor", "double T = (fh[3] - (fh[1] * fh[1] + fh[2] * fh[2]) / rho) / (p->b * rho);",
     "double T = (fh[3] - (fh[1] * fh[1] + fh[2] * fh[2]) / rho) / (2.0 * p->b * rho);"),
    ("mc_breakpoint", "if (theta <= 1.0 / 3.0) return 2.0 * theta;", "if (theta <= 1.0 / 2.0) return 2.0 * theta;"),
    ("minmod_cap", "if (theta <= 1.0) return theta;", "if (theta <= 1.0) return 1.0;"),
    ("matrix_row_12_index", "out[11] = cx * dxy;", "out[11] = cy * dxy;"),
    ("matrix_row_14_term", "out[13] = c2 * ce;", "out[13] = ce * ce;"),
    ("eta_on_wrong_group", "C->eta[i] = (g == 0) ? eta0 : 0.0;", "C->eta[i] = (g == 1) ? eta0 : 0.0;"),
    ("wall_density", "double rw = r1 * T1 / st[3];", "double rw = r1;"),
    ("wall_velocity_ignored", "feq_velocity(C, p->b, rw, st[1], st[2], st[3], eqw);",
     "feq_velocity(C, p->b, rw, u1x, u1y, st[3], eqw);"),
    ("wall_nonequilibrium_dropped", "for (int i = 0; i < Q; ++i) fw[i] = eqw[i] + (f1[i] - eq1[i]);",
     "for (int i = 0; i < Q; ++i) fw[i] = eqw[i] + 0.0 * (f1[i] - eq1[i]);"),
    ("wall_ghosts_constant", "for (int i = 0; i < Q; ++i) gk[i] = (k + 1) * fw[i] - k * f1[i];",
     "for (int i = 0; i < Q; ++i) gk[i] = fw[i] + 0.0 * k * f1[i];"),
    ("outflow_x_copies_second_node", "load_node(g, side == 0 ? 0 : nx - 1, y, tmp);",
     "load_node(g, side == 0 ? 1 : nx - 2, y, tmp);"),
    ("outflow_y_copies_second_node", "load_node(g, x, side == 2 ? 0 : ny - 1, tmp);",
     "load_node(g, x, side == 2 ? 1 : ny - 2, tmp);"),
    ("equilibrium_x_velocity_swapped", EQX, EQX.replace("st[1], st[2], st[3], eq", "st[2], st[1], st[3], eq")),
    ("gradient_x_uses_dy", "double duxdx = (ux[UIX(x + 1, y)] - ux[UIX(x - 1, y)]) / (2.0 * p->dx);",
     "double duxdx = (ux[UIX(x + 1, y)] - ux[UIX(x - 1, y)]) / (2.0 * p->dy);"),
    ("courant_spacings_swapped", "double nu = p->dt / (C->A[i] * ((a == 0) ? p->dx : p->dy));",
     "double nu = p->dt / (C->A[i] * ((a == 0) ? p->dy : p->dx));"),
    ("noneq_star_relative_velocity_sign", STAR, STAR.replace("C.vx[i] - vx", "C.vx[i] + vx")),
    ("noneq_star_components_swapped", STAR, STAR.replace("C.vx[i] - vx, C.vy[i] - vy", "C.vy[i] - vy, C.vx[i] - vx")),
    ("noneq_star_eta_dropped", STAR, STAR.replace("C.eta[i], row", "0.0, row")),
    ("noneq_without_equilibrium", "for (int i = 0; i < Q; ++i) gneq[i] = fl[i] - fe[i];",
     "for (int i = 0; i < Q; ++i) gneq[i] = fl[i] - 0.0 * fe[i];"),
    ("mc_cap", "        return 2.0;\n    case ORC_LIM_MINMOD:", "        return 1.0;\n    case ORC_LIM_MINMOD:"),
    ("mc_middle_half_dropped", "if (theta <= 3.0) return (1.0 + theta) / 2.0;",
     "if (theta <= 3.0) return (1.0 + theta);"),
    ("theta_inverted", "double theta = (f0 - fm) / den;",
     "double theta = (f0 - fm) == 0.0 ? 1e300 : den / (f0 - fm);"),
    ("courant_factor_sign", FACES, FACES.replace("(1.0 - nu)", "(1.0 + nu)")),
    ("relaxation_skips_first_nonconserved", "for (int k = 4; k < Q; ++k) R[k] = p->s[k] * (fh[k] - fe[k]);",
     "for (int k = 5; k < Q; ++k) R[k] = p->s[k] * (fh[k] - fe[k]);"),
    ("correction_ratio_inverted", "double k8 = p->s[7] / p->s[4] - 1.0;", "double k8 = p->s[4] / p->s[7] - 1.0;"),
    ("collision_transposed", "for (int k = 0; k < Q; ++k) coll += C->Minv[i][k] * R[k];",
     "for (int k = 0; k < Q; ++k) coll += C->Minv[k][i] * R[k];"),
    ("collision_sign", "fnew[i] = f[i] - conv - p->dt * coll;", "fnew[i] = f[i] - conv + p->dt * coll;"),
    ("feq_13_pressure_sign", "out[12] = (-2.0 * P + jx", "out[12] = (2.0 * P + jx"),
    ("feq_14_b_coefficient", "(6.0 + b) * T * j2", "(4.0 + b) * T * j2"),
    ("feq_16_b_coefficient", "out[15] = ((b + 4.0) * P", "out[15] = ((b + 2.0) * P"),
    ("energy_with_b_fixed_at_2", "double e = rho * (b * T + ux * ux + uy * uy);",
     "double e = rho * (2.0 * T + ux * ux + uy * uy);"),
]

# the pins, cheapest first
PINS = [
    lambda o: T_const.test_velocity_set_matches_paper(o),
    lambda o: T_const.test_inverse(o),
    lambda o: T_const.test_first_rows_are_conserved_moments(o),
    lambda o: T_const.test_seven_moment_relations(o, 5.0),
    lambda o: T_const.test_feq_hat_consistent_with_velocity_space(o),
    lambda o: T_const.test_eta_enters_only_through_m(o),
    lambda o: T_inv.test_uniform_state_is_fixed_point(o),
    lambda o: T_inv.test_walls_hold_a_matching_uniform_state(o, "y"),
    lambda o: T_inv.test_walls_hold_a_matching_uniform_state(o, "x"),
    lambda o: T_inv.test_conservation_periodic(o, "mc"),
    lambda o: T_inv.test_rotation_symmetry(o),
    lambda o: T_inv.test_rotation_symmetry_with_unequal_spacings(o),
    lambda o: T_inv.test_mirror_symmetry(o),
    lambda o: T_inv.test_boundaries_do_not_act_ahead_of_waves(o),
    lambda o: T_inv.test_ghosts_act_as_the_lines_they_stand_for(o, "outflow", "x"),
    lambda o: T_inv.test_ghosts_act_as_the_lines_they_stand_for(o, "outflow", "y"),
    lambda o: T_inv.test_ghosts_act_as_the_lines_they_stand_for(o, "equilibrium", "x"),
    lambda o: T_inv.test_ghosts_act_as_the_lines_they_stand_for(o, "equilibrium", "y"),
    lambda o: T_noneq.test_zero_at_equilibrium(o),
    lambda o: T_noneq.test_star_equals_plain_at_rest(o),
    lambda o: T_noneq.test_conserved_components_vanish(o),
    lambda o: T_noneq.test_central_moment_shift_identities(o),
    lambda o: T_text.test_unit_courant_is_exact_shift(o),
    lambda o: T_text.test_unit_courant_is_exact_shift_with_unequal_spacings(o),
    lambda o: T_text.test_reduces_to_textbook_limited_scheme(o, "lw"),
    lambda o: T_text.test_reduces_to_textbook_limited_scheme(o, "minmod"),
    lambda o: T_text.test_reduces_to_textbook_limited_scheme(o, "mc"),
    lambda o: T_text.test_total_variation_diminishing(o, "mc"),
    lambda o: T_phys.test_shear_wave_decay_rate_uses_s7(o),
    lambda o: T_phys.test_sod_vs_exact(o, "mc"),
    lambda o: T_phys.test_thermal_wave_decay_rate_uses_s8_s9(o),
    lambda o: T_phys.test_couette_profiles_and_prandtl_effect(o),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_a_pin_catches_the_planted_mistake(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path_c = tmp_path / f"{name}.c"
    path_so = tmp_path / f"lib{name}.so"
    path_c.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(path_so), str(path_c), "-lm"])
    saved = oracle._load()
    oracle._lib = oracle.open_library(str(path_so))
    caught = None
    try:
        for k, pin in enumerate(PINS):
            try:
                pin(oracle)
            except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError):
                caught = k
                break
    finally:
        oracle._lib = saved
    assert caught is not None, f"no pin catches the planted mistake {name}"
