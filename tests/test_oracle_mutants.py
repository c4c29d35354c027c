"""Mutation check of the oracle's pins: each case plants one plausible mistake in a copy
of the oracle source (CPU only), builds it, and requires that at least one pin fails
against the broken copy."""
import os

import pytest

import tests.test_oracle as pins
from oracle import lbaref

SRC = open(os.path.join(os.path.dirname(lbaref.__file__), "lbaref.c")).read()

# (name, original text, planted text, pins expected to catch it)
MUTANTS = [
    ("residual_sign", "e[0] = P->obs_z[i] - pi[0];", "e[0] = pi[0] - P->obs_z[i];",
     [lambda: pins.test_gradient_equals_minus_two_b(lbaref, 0)]),
    ("stereo_jacobian_row", "-(P->fx * Xc[0] - P->bf) * iz2", "-(P->fx * Xc[0] + P->bf) * iz2",
     [lambda: pins.test_jacobians_central_differences(lbaref, True)]),
    ("stereo_projection", "pi[2] = stereo ? pi[0] - P->bf * iz : 0.0;",
     "pi[2] = stereo ? pi[0] + P->bf * iz : 0.0;",
     [lambda: pins.test_projection_golden(lbaref)]),
    ("huber_weight", "*w = d / rs;", "*w = 1.0;",
     [lambda: pins.test_huber_golden(lbaref)]),
    ("huber_cost", "*rho = 2.0 * d * rs - d2;", "*rho = d * rs;",
     [lambda: pins.test_huber_weight_is_derivative_and_continuous(lbaref)]),
    ("information_weight", "double om = w / P->sigma2[P->obs_oct[i]];\n        for (int a = 0; a < 3; ++a) {",
     "double om = w;\n        for (int a = 0; a < 3; ++a) {",
     [lambda: pins.test_gradient_equals_minus_two_b(lbaref, 1)]),
    ("point_damping_missing",
     "for (int q = 0; q < 9; ++q) V[q] = B->Hll[j * 9 + q] + ((q % 4 == 0) ? lambda : 0.0);\n        if (inv3_spd(V, Vi)) return 1;\n        for (int ia",
     "for (int q = 0; q < 9; ++q) V[q] = B->Hll[j * 9 + q] + ((q % 4 == 0) ? 0.5 * lambda : 0.0);\n        if (inv3_spd(V, Vi)) return 1;\n        for (int ia",
     [lambda: pins.test_schur_step_equals_dense_solve(lbaref, 0, 4, 1, 20)]),
    ("backsub_transposed_W", "rhs[c] -= B->W[ia * 18 + a * 3 + c] * dp[ka * 6 + a];",
     "rhs[c] -= B->W[ia * 18 + (a % 3) * 6 + c] * dp[ka * 6 + a];",
     [lambda: pins.test_schur_step_equals_dense_solve(lbaref, 0, 4, 1, 20)]),
    ("schur_rhs_sign", "r[ka * 6 + a] -= acc;", "r[ka * 6 + a] += acc;",
     [lambda: pins.test_schur_step_equals_dense_solve(lbaref, 1, 5, 2, 30)]),
    ("exp_coefficient", "*B = 2.0 * h * h / (th * th);", "*B = h * h / (th * th);",
     [lambda: pins.test_se3_exp_matches_scipy_expm(lbaref, 0.3)]),
    ("left_jacobian_coupling", "c2 * (WWU[i] + UWW[i] - 3.0 * WUW[i])", "c2 * (WWU[i] + UWW[i] + 3.0 * WUW[i])",
     [lambda: pins.test_se3_left_jacobian_finite_difference(lbaref, 0.8)]),
    ("cholesky_index", "sum -= A[i * n + k] * A[j * n + k];", "sum -= A[i * n + k] * A[k * n + j];",
     [lambda: pins.test_cholesky_matches_numpy(lbaref)]),
    ("gain_denominator", "den += dp[q] * (lambda * dp[q] + B->bp[q]);",
     "den += dp[q] * (lambda * dp[q] - B->bp[q]);",
     [lambda: pins.test_noise_free_converges_to_ground_truth(lbaref, pins.synth.c1_mono)]),
    ("outlier_threshold_swapped", "double th = P->obs_type[i] ? O->chi2_stereo : O->chi2_mono;",
     "double th = P->obs_type[i] ? O->chi2_mono : O->chi2_stereo;",
     [lambda: pins.test_outlier_flags_recomputed_from_states(lbaref)]),
    ("pose_retraction_right", "T2[12 * k + r * 4 + 3] = R[r * 3 + 0] * T[12 * k + 3] + R[r * 3 + 1] * T[12 * k + 7] +\n                                     R[r * 3 + 2] * T[12 * k + 11] + t[r];",
     "T2[12 * k + r * 4 + 3] = T[12 * k + r * 4 + 3] + t[r];",
     [lambda: pins.test_noise_free_converges_to_ground_truth(lbaref, pins.synth.c1_mono)]),
    ("grad_z_sign", "g_z[q * P->n_obs + i] = q < r ? 2.0 * om * e[q] : 0.0;",
     "g_z[q * P->n_obs + i] = q < r ? -2.0 * om * e[q] : 0.0;",
     [lambda: pins.test_cost_gradient_finite_differences(lbaref, 0.0)]),
    # the damping schedule
    ("nielsen_square_not_cube", "*lambda *= fmax(1.0 / 3.0, 1.0 - f * f * f);",
     "*lambda *= fmax(1.0 / 3.0, 1.0 - f * f);",
     [lambda: pins.test_damping_update_golden(lbaref)]),
    ("nu_not_reset_on_accept", "        *nu = 2.0;\n    } else {", "        (void)0;\n    } else {",
     [lambda: pins.test_damping_update_golden(lbaref)]),
    ("reject_times_three", "*lambda *= *nu;", "*lambda *= 3.0;",
     [lambda: pins.test_damping_update_golden(lbaref)]),
    ("lambda0_pose_blocks_only", "for (int a = 0; a < 3; ++a) md = fmax(md, B->Hll[j * 9 + a * 4]);",
     "for (int a = 0; a < 3; ++a) md = fmax(md, 0.0 * B->Hll[j * 9 + a * 4]);",
     [lambda: pins.test_initial_damping_each_round(lbaref, "points_only")]),
    ("no_round2_reinit",
     [("double lambda = lbaref_initial_damping(O->tau, B->maxdiag), nu = 2.0;",
       "static double carry = -1.0;\n    double lambda = (round == 2 && carry >= 0.0) ? carry : "
       "lbaref_initial_damping(O->tau, B->maxdiag), nu = 2.0;"),
      ("*lambda_out = lambda;", "*lambda_out = lambda;\n    carry = lambda;")],
     None,
     [lambda: pins.test_initial_damping_each_round(lbaref, "posed")]),
    ("termination_off_by_one", "for (int trial = 0; trial < O->max_trials; ++trial) {",
     "for (int trial = 0; trial <= O->max_trials; ++trial) {",
     [lambda: pins.test_rejections_end_round_after_max_trials(lbaref)]),
]


def _plant(name, orig, planted):
    """The oracle source with one mistake planted: `orig` is one anchor text replaced by
    `planted`, or a list of (anchor, replacement) pairs applied together."""
    edits = orig if isinstance(orig, list) else [(orig, planted)]
    src = SRC
    for a, b in edits:
        assert src.count(a) == 1, f"mutation anchor for {name} not unique in the oracle source"
        src = src.replace(a, b)
    return src


@pytest.mark.parametrize("name,orig,planted,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, orig, planted, checks):
    path = lbaref.build_variant(_plant(name, orig, planted), str(tmp_path / f"mut_{name}.so"))
    caught = False
    with lbaref.use_library(path):
        for chk in checks:
            try:
                chk()
            except AssertionError:
                caught = True
    assert caught, f"planted mistake {name} passed every pin"
