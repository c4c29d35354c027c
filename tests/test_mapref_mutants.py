"""Mutation check of the pins of the local-mapping search oracle: each case plants one
plausible mistake in a copy of its source (CPU only), builds it, and requires that at
least one pin fails against the broken copy."""
import os

import pytest

import tests.test_mapref_oracle as pins
from oracle import mapref

SRC = open(os.path.join(os.path.dirname(mapref.__file__), "mapref.c")).read()

C_ANCHOR = "                    if (d > P->th_low || d >= bd) continue;\n                    const int o = S->kp_oct[j];"
F_ANCHOR = "                if (d > P->th_low || d >= bd) continue;\n                best = j;"

MUTANTS = [
    ("fundamental_transposed", "const double l0 = (F[0] * ua + F[1] * va) + F[2];\n    const double l1 = (F[3] * ua + F[4] * va) + F[5];\n    const double l2 = (F[6] * ua + F[7] * va) + F[8];",
     "const double l0 = (F[0] * ua + F[3] * va) + F[6];\n    const double l1 = (F[1] * ua + F[4] * va) + F[7];\n    const double l2 = (F[2] * ua + F[5] * va) + F[8];",
     ["test_epipolar_distance_is_zero_for_a_point_seen_twice"]),
    ("relative_rotation_order", "mul33(Rb, RaT, R);", "mul33(RaT, Rb, R);",
     ["test_epipolar_distance_is_zero_for_a_point_seen_twice"]),
    ("essential_sign", "const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};",
     "const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], t[1], t[0], 0.0};",
     ["test_epipolar_distance_is_zero_for_a_point_seen_twice"]),
    ("hamming_31_bits", "for (int bit = 0; bit < 32; ++bit)", "for (int bit = 0; bit < 31; ++bit)",
     ["test_hamming_matches_numpy_bit_count"]),
    ("corr_tie_to_larger_index", C_ANCHOR,
     C_ANCHOR.replace("d >= bd", "d > bd"), ["test_correspondence_planted_cases"]),
    ("corr_threshold_strict", C_ANCHOR,
     C_ANCHOR.replace("d > P->th_low", "d >= P->th_low"), ["test_correspondence_planted_cases"]),
    ("corr_sigma_of_searching_keypoint", "if (e2 < 0.0 || !(e2 < P->epi_chi2 * S->sigma2[o])) continue;",
     "if (e2 < 0.0 || !(e2 < P->epi_chi2 * S->sigma2[S->kp_oct[i]])) continue;",
     ["test_correspondence_epipolar_tolerance_scales_with_the_neighbour_octave"]),
    ("corr_epipole_test_for_stereo", "if (mono_a && S->kp_ur[j] < 0.0f) {", "if (1) {",
     ["test_correspondence_epipole_test_only_between_monocular_keypoints"]),
    ("corr_epipole_uses_scale_squared", "if (dx * dx + dy * dy < P->epipole_min * S->scale[o]) continue;",
     "if (dx * dx + dy * dy < P->epipole_min) continue;",
     ["test_correspondence_epipole_test_only_between_monocular_keypoints"]),
    ("corr_free_flag_of_neighbour_ignored", "                    if (!S->kp_free[j]) continue;\n", "",
     ["test_correspondence_planted_cases"]),
    ("resolution_tie_to_larger_index", "(dout[k] == dout[i] && k < i)", "(dout[k] == dout[i] && k > i)",
     ["test_correspondence_deferred_resolution"]),
    ("fuse_octave_window", "if (o < level - 1 || o > level) continue;", "if (o < level || o > level + 1) continue;",
     ["test_fusion_planted_cases"]),
    ("fuse_stereo_threshold", "if (e2 > P->chi2_stereo * S->sigma2[o]) continue;",
     "if (e2 > P->chi2_mono * S->sigma2[o]) continue;",
     ["test_fusion_stereo_reprojection_uses_the_right_coordinate"]),
    ("fuse_right_coordinate_ignored", "const double e2 = (ex * ex + ey * ey) + er * er;",
     "const double e2 = (ex * ex + ey * ey) + 0.0 * er;",
     ["test_fusion_stereo_reprojection_uses_the_right_coordinate"]),
    ("fuse_viewing_angle_45", "dot * dot < 0.25 * d2", "dot * dot < 0.5 * d2", ["test_fusion_geometric_gates"]),
    ("fuse_radius_not_scaled", "const double radius = P->radius_th * S->scale[level];",
     "const double radius = P->radius_th;", ["test_fusion_planted_cases"]),
    ("fuse_tie_to_larger_index", F_ANCHOR, F_ANCHOR.replace("d >= bd", "d > bd"), ["test_fusion_planted_cases"]),
    ("fuse_level_one_less", "while (level < S->n_levels - 1 && S->scale[level] * S->scale[level] * d2 < dmax[p] * dmax[p]) ++level;",
     "while (level < S->n_levels - 1 && S->scale[level + 1] * S->scale[level + 1] * d2 < dmax[p] * dmax[p]) ++level;",
     ["test_fusion_planted_cases"]),
    ("fuse_skip_ignored", "            if (skip && skip[o_idx]) continue;\n", "", ["test_fusion_planted_cases"]),
    ("cull_self_counted", "if (b == a || obs_pt[b] != obs_pt[a] || (active && !active[b])) continue;",
     "if (obs_pt[b] != obs_pt[a] || (active && !active[b])) continue;", ["test_culling_hand_worked_example"]),
    ("cull_strictly_above", "(int64_t)den * kf_red[k] >= (int64_t)num * kf_obs[k]",
     "(int64_t)den * kf_red[k] > (int64_t)num * kf_obs[k]", ["test_culling_threshold_is_at_least_ninety_percent"]),
    ("cull_slack_ignored", "if (obs_oct[b] <= obs_oct[a] + slack) ++others;", "if (obs_oct[b] <= obs_oct[a]) ++others;",
     ["test_culling_hand_worked_example"]),
]


@pytest.mark.parametrize("name,orig,planted,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, orig, planted, checks):
    assert SRC.count(orig) == 1, f"mutation anchor for {name} not unique in the oracle source"
    path = mapref.build_variant(SRC.replace(orig, planted), str(tmp_path / f"mut_{name}.so"))
    store = pins.synth.keyframe_store(seed=11, K=12, M=4000, kp_per_kf=400, walk_length=3.0)
    caught = False
    with mapref.use_library(path):
        for chk in checks:
            fn = getattr(pins, chk)
            args = {"mref": mapref}
            if "store" in fn.__code__.co_varnames[:fn.__code__.co_argcount]:
                args["store"] = store
            try:
                fn(**args)
            except AssertionError:
                caught = True
    assert caught, f"planted mistake {name} passed every pin"
