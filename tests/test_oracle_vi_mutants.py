"""Mutation check of the stereo-inertial oracle's pins: each case plants one plausible
mistake in a copy of the oracle source (CPU only), builds it, and requires that at least
one pin of tests/test_oracle_vi.py fails against the broken copy."""
import os

import pytest

import tests.test_oracle_vi as pins
from oracle import lbaref

SRC = open(os.path.join(os.path.dirname(lbaref.__file__), "lbaref.c")).read()

MUTANTS = [
    ("gravity_sign_velocity", "q->u[a] = V[3 * j + a] - V[3 * i + a] - I->g[a] * dt;",
     "q->u[a] = V[3 * j + a] - V[3 * i + a] + I->g[a] * dt;",
     [lambda: pins.test_residual_is_zero_at_the_true_states(lbaref)]),
    ("half_gravity_factor", "- 0.5 * I->g[a] * dt * dt;", "- I->g[a] * dt * dt;",
     [lambda: pins.test_residual_is_zero_at_the_true_states(lbaref)]),
    ("bias_correction_sign", "q->r[3 + a] = Ru[a] - (I->dv[3 * e + a] + a1[a] + a2[a]);",
     "q->r[3 + a] = Ru[a] - (I->dv[3 * e + a] - a1[a] + a2[a]);",
     [lambda: pins.test_residual_is_zero_at_the_true_states(lbaref)]),
    ("rotation_residual_order", "matmul(dRcT, RiTRj, q->E, 3, 3, 3);", "matmul(RiTRj, dRcT, q->E, 3, 3, 3);",
     [lambda: pins.test_residual_is_zero_at_the_true_states(lbaref),
      lambda: pins.test_jacobian_blocks_match_central_differences(lbaref)]),
    ("lever_arm_missing", "matmul(RcwT, tx, Ptw, 3, 3, 3);", "memset(Ptw, 0, sizeof(Ptw));",
     [lambda: pins.test_jacobian_blocks_match_central_differences(lbaref)]),
    ("jr_inverse_as_identity", "lbaref_so3_jr_inv(q.r, Jri);",
     "for (int z = 0; z < 9; ++z) Jri[z] = (z % 4 == 0) ? 1.0 : 0.0;",
     [lambda: pins.test_jacobian_blocks_match_central_differences(lbaref)]),
    ("velocity_bias_jacobian_sign", "for (int a = 0; a < 9; ++a) M[a] = -I->J_vg[9 * e + a];",
     "for (int a = 0; a < 9; ++a) M[a] = I->J_vg[9 * e + a];",
     [lambda: pins.test_jacobian_blocks_match_central_differences(lbaref)]),
    ("position_velocity_dt", "for (int a = 0; a < 9; ++a) M[a] = -RiT[a] * dt;",
     "for (int a = 0; a < 9; ++a) M[a] = -RiT[a];",
     [lambda: pins.test_jacobian_blocks_match_central_differences(lbaref)]),
    ("jr_coefficient_sign", "Jr[i] = ((i % 4 == 0) ? 1.0 : 0.0) - B * W[i] + C * W2[i];",
     "Jr[i] = ((i % 4 == 0) ? 1.0 : 0.0) + B * W[i] + C * W2[i];",
     [lambda: pins.test_right_jacobian_and_its_inverse(lbaref)]),
    ("log_near_pi_axis", "for (int q = 0; q < 3; ++q) a[q] = Bm[q * 3 + k];",
     "for (int q = 0; q < 3; ++q) a[q] = R[q * 3 + k] + (q == k ? 1.0 : 0.0);",
     [lambda: pins.test_so3_log_matches_scipy_rotation_vectors(lbaref)]),
    ("no_damping_on_velocity_and_bias", "if (a % 15 >= 6) S[a * n + a] += lambda;", "(void)0;",
     [lambda: pins.test_schur_step_equals_dense_step(lbaref, 7, 10.0)]),
    ("velocity_step_dropped", "V2[3 * k + a] = S->V[3 * k + a] + (ok >= 0 ? d[15 * ok + 6 + a] : 0.0);",
     "V2[3 * k + a] = S->V[3 * k + a];",
     [lambda: pins.test_noise_free_window_converges_to_the_truth(lbaref)]),
    ("denominator_without_inertial_gradient", "double g = bi[15 * k + a] + (a < 6 ? B->bp[6 * k + a] : 0.0);",
     "double g = (a < 6 ? B->bp[6 * k + a] : 0.0);",
     [lambda: pins.test_predicted_decrease_matches_the_dense_model(lbaref)]),
    ("inertial_gradient_sign", "b[ga] -= g;", "b[ga] += g;",
     [lambda: pins.test_schur_step_equals_dense_step(lbaref, 6, 1e-3),
      lambda: pins.test_noise_free_window_converges_to_the_truth(lbaref)]),
    ("lambda0_without_inertial_diagonal", "double v = Hi[(15 * k + a) * n + 15 * k + a];",
     "double v = 0.0 * Hi[(15 * k + a) * n + 15 * k + a];",
     [lambda: pins.test_initial_damping_includes_the_inertial_blocks(lbaref)]),
]


@pytest.mark.parametrize("name,orig,planted,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, orig, planted, checks):
    assert SRC.count(orig) == 1, f"mutation anchor for {name} not unique in the oracle source"
    path = lbaref.build_variant(SRC.replace(orig, planted), str(tmp_path / f"mut_{name}.so"))
    caught = False
    with lbaref.use_library(path):
        for chk in checks:
            try:
                chk()
            except AssertionError:
                caught = True
    assert caught, f"planted mistake {name} passed every pin"
