"""Planted mistakes: each mutation below edits a copy of the oracle's C source
(on the CPU only), rebuilds it, and requires that at least one pin of
test_oracle_pins.py fails against the mutant.  This checks that the pins are
strong enough to catch a dropped term, a wrong sign, index or operand."""
import os
import shutil
import subprocess

import pytest

import oracle
import synth
from tests import test_oracle_pins as pins
from tests import test_oracle_map as mapt
from tests import test_oracle_motion as motion
from tests import test_oracle_orb as orb
from tests import test_oracle_pyramid as pyr

HERE = os.path.dirname(os.path.abspath(oracle.__file__))

MUTANTS = {
    "hamming_and": ("a[q] ^ b[q]", "a[q] & b[q]"),
    "sad_no_centre": ("(int)IL[(size_t)(sv + dy) * Wl + su + dx] - cL", "(int)IL[(size_t)(sv + dy) * Wl + su + dx]"),
    "sad_shift_sign": ("su0 + k + dx]", "su0 - k + dx]"),
    "subpixel_sign": ("(float)(a - e)", "(float)(e - a)"),
    "subpixel_den": ("2 * (a + e - 2 * c)", "(a + e - 2 * c)"),
    "median_index": ("v[n / 2]", "v[(n - 1) / 2]"),
    "median_ratio": ("(int64_t)den * sad[i] < (int64_t)num * m", "(int64_t)num * sad[i] < (int64_t)den * m"),
    "pinhole_level_window": ("oj < oi - lw ||", "oj < oi - lw - 1 ||"),
    "pinhole_disp_sign": ("float disp = xL[i] - uR;", "float disp = uR - xL[i];"),
    "pinhole_band": ("floorf(yR[j] - r)", "floorf(yR[j] + r)"),
    "pinhole_th_orb": ("!(best_h < th_orb)", "!(best_h <= th_orb)"),
    "pinhole_depth": ("cd[i] = bf / disp;", "cd[i] = disp / bf;"),
    "kb_distort_term": ("return th * ((((1.0 + k1 * t2) + k2 * t4)", "return th * ((((1.0 + k1 * t2) + k2 * t2)"),
    "kb_unproject_tan": ("tan(th) / thd", "sin(th) / thd"),
    "kb_newton_deriv": ("(1.0 + 3.0 * k1 * t2)", "(1.0 + 2.0 * k1 * t2)"),
    "tri_transpose": ("Rrl[r][c] = (double)R_lr[3 * c + r];", "Rrl[r][c] = (double)R_lr[3 * r + c];"),
    "tri_t_sign": ("trl[r] = -(((Rrl", "trl[r] = (((Rrl"),
    "fish_ratio": ("ratio_den * h1 < ratio_num * h2", "ratio_num * h1 < ratio_den * h2"),
    "fish_second": ("if (h < h1) { h2 = h1; h1 = h; j1 = j; }", "if (h < h1) { h1 = h; j1 = j; }"),
    "search_R_transpose": ("((R[0] * X + R[1] * Y) + R[2] * Z)", "((R[0] * X + R[3] * Y) + R[6] * Z)"),
    "search_radius_swap": ("(vcos > cos_narrow ? r_narrow : r_wide)", "(vcos > cos_narrow ? r_wide : r_narrow)"),
    "search_uR_sign": ("uR = u - bf * (1.0f / zc)", "uR = u + bf * (1.0f / zc)"),
    "search_preassigned_ignored": ("if (preassigned && preassigned[k]) continue;", ""),
    "search_level_hi": ("ok > pred + lv_hi", "ok > pred + lv_hi + 1"),
    "search_second_level": ("else if (h < b2) { b2 = h; l2 = ok; }", "else if (h < b2) { b2 = h; }"),
    "search_window_y": ("fabsf(ky[k] - v) < Rm", "fabsf(ky[k] - u) < Rm"),
    "search_dist_hi": ("dist <= hi", "dist <= lo"),
    "predict_level_off_by_one": ("if (sf[l] >= ratio) return l;", "if (sf[l] >= ratio) return l + 1 < n_levels ? l + 1 : l;"),
    # visibility tests of the search (each must reject its own cases)
    "search_dist_lo_dropped": ("if (!(dist >= lo)) { ++n_near; continue; }", ""),
    "search_dist_lo_strict": ("if (!(dist >= lo))", "if (!(dist > lo))"),
    "search_dist_hi_strict": ("if (!(dist <= hi))", "if (!(dist < hi))"),
    "search_viewcos_dropped": ("if (!(vcos >= cos_lim)) { ++n_angle; continue; }", ""),
    "search_viewcos_strict": ("if (!(vcos >= cos_lim))", "if (!(vcos > cos_lim))"),
    "search_viewcos_no_divide": (") / dist;\n        if (!(vcos", ");\n        if (!(vcos"),
    # triangulation check of fisheye pairs
    "fish_parallax_dropped": ("if (!(cosp <= cos_max)) { ++n_par; continue; }", ""),
    "fish_left_depth_dropped": ("if (!(X[2] > 0.0)) { ++n_dep; continue; }", ""),
    "fish_right_depth_dropped": ("if (!(X2[2] > 0.0)) { ++n_dep; continue; }", ""),
    "fish_right_reproj_left_level": ("chi2 * (double)sigma2[oR[j1]]", "chi2 * (double)sigma2[oL[i]]"),
    "fish_right_reproj_half_bound": ("chi2 * (double)sigma2[oR[j1]]", "0.5 * chi2 * (double)sigma2[oR[j1]]"),
    "fish_left_reproj_right_level": ("chi2 * (double)sigma2[oL[i]]", "chi2 * (double)sigma2[oR[j1]]"),
    "fish_right_reproj_dropped": ("if (!(ex * ex + ey * ey <= chi2 * (double)sigma2[oR[j1]])) { ++n_rep; continue; }", ""),
    "fish_one_target_enough": ("if (nT < 2) continue;", "if (nT < 1) continue;"),
    "pyramid_no_centre_alignment": ("(int64_t)(2 * x + 1) * n_in - n_out", "(int64_t)(2 * x) * n_in"),
    "pyramid_weight_rounded": ("(256 * r) / den", "(256 * r + den / 2) / den"),
    "pyramid_result_truncated": ("(v + 32768) >> 16", "v >> 16"),
    "pyramid_size_truncated": ("w[l] = (int32_t)floorf(fw + 0.5f);", "w[l] = (int32_t)floorf(fw);"),
    "pyramid_rows_from_width": ("pyramid_tap(y, H, h[l], &y0, &b);", "pyramid_tap(y, W, h[l], &y0, &b);"),
    "pyramid_weights_swapped": ("const int top = (256 - a) * p00 + a * p01;", "const int top = a * p00 + (256 - a) * p01;"),
    "last_forward_window": ("if (direction > 0) { lv_min = ol; lv_max = n_levels - 1; }",
                            "if (direction > 0) { lv_min = ol + 1; lv_max = n_levels - 1; }"),
    "last_backward_window": ("else if (direction < 0) { lv_min = 0; lv_max = ol; }",
                             "else if (direction < 0) { lv_min = 0; lv_max = ol - 1; }"),
    "last_radius_level": ("const float r = th * sf[ol < n_levels ? ol : n_levels - 1];", "const float r = th * sf[0];"),
    "last_threshold_strict": ("if (kbest < 0 || !(best <= th_high)) continue;", "if (kbest < 0 || !(best < th_high)) continue;"),
    "last_stereo_gate_sign": ("if (u_right) ur_proj = u - bf * (1.0f / zc);", "if (u_right) ur_proj = u + bf * (1.0f / zc);"),
    "last_conflict_skipped": ("    resolve_conflicts(nL, cand_k, cand_h, nK, alive);\n", ""),
    "rotation_sign": ("float rot = a_last - a_cur;", "float rot = a_cur - a_last;"),
    "rotation_wrap": ("int bin = (int)roundf(rot * factor) % bins;", "int bin = (int)roundf(rot * factor); if (bin >= bins) bin = bins - 1;"),
    "three_fullest_tenth": ("if (10 * m2 < m1) { i2 = -1; i3 = -1; }", "if (2 * m2 < m1) { i2 = -1; i3 = -1; }"),
    "three_fullest_third_always": ("else if (10 * m3 < m1) i3 = -1;", ""),
    "three_fullest_tie_to_later": ("if (c > m1) { m3 = m2;", "if (c >= m1) { m3 = m2;"),
    "map_pair_from_the_end": ("int h = 0, src = n1;", "int h = 0, src = n1 + 1;"),
    "map_append_at_old_count": ("map_copy(pos, normal, dmin, dmax, desc, n1 + j, ipos", "map_copy(pos, normal, dmin, dmax, desc, n + j, ipos"),
    "map_duplicates_accepted": ("if (r < 0 || r >= n || gone[r])", "if (r < 0 || r >= n)"),
    "map_normal_not_moved": ("        normal[3 * to + c] = snormal[3 * from + c];\n", ""),
    "map_capacity_strict": ("if ((int64_t)n1 + n_insert > capacity)", "if ((int64_t)n1 + n_insert >= capacity)"),
    "orb_ring_offset": ("orb_ring_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1}",
                        "orb_ring_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -2}"),
    "orb_arc_of_eight": ("for (int k = 0; k < 9; ++k) {\n            const int r = (a + k) % 16;",
                         "for (int k = 0; k < 8; ++k) {\n            const int r = (a + k) % 16;"),
    "orb_score_not_minus_one": ("if (lo_dark - 1 > best) best = lo_dark - 1;", "if (lo_dark > best) best = lo_dark;"),
    "orb_threshold_strict": ("if (s >= t) v = s;", "if (s > t) v = s;"),
    "orb_window_right_edge": ("x < w - edge &&", "x <= w - edge &&"),
    "orb_nms_keeps_ties": ("if (v <= nb) keep = 0;", "if (v < nb) keep = 0;"),
    "orb_nms_four_neighbours": ("if (dx == 0 && dy == 0) continue;\n                        const int nx",
                                "if (dx == dy || dx == -dy) continue;\n                        const int nx"),
    "orb_coordinates_unscaled": ("x[n] = (float)xx * sf[l];", "x[n] = (float)xx * sf[0];"),
    "orb_blur_unrounded": ("(uint8_t)((acc + 2048) >> 12)", "(uint8_t)(acc >> 12)"),
    "orb_blur_weights": ("orb_blur_k[7] = {1, 6, 15, 20, 15, 6, 1}", "orb_blur_k[7] = {2, 6, 15, 18, 15, 6, 2}"),
    "orb_disc_strict": ("if (dx * dx + dy * dy > 225) continue;", "if (dx * dx + dy * dy >= 225) continue;"),
    "orb_m01_sign": ("m01 += (int64_t)dy * I;", "m01 -= (int64_t)dy * I;"),
    "orb_turn_sign": ("c1 = orb_round_ratio((int64_t)x1 * m10 - (int64_t)y1 * m01, m2);",
                      "c1 = orb_round_ratio((int64_t)x1 * m10 + (int64_t)y1 * m01, m2);"),
    "orb_bit_order": ("d[t / 8] |= (uint8_t)(1u << (t % 8));", "d[t / 8] |= (uint8_t)(0x80u >> (t % 8));"),
    "orb_test_reversed": ("if (B[(size_t)(v + r1) * W + (u + c1)] < B[", "if (B[(size_t)(v + r1) * W + (u + c1)] > B["),
    "orb_descriptor_unsmoothed": ("const uint8_t *B = blurred + off[l];", "const uint8_t *B = pyr + off[l];"),
    "orb_orientation_smoothed": ("const uint8_t *img = pyr + off[l];\n        const uint8_t *B",
                                 "const uint8_t *img = blurred + off[l];\n        const uint8_t *B"),
    "conflict_tie": ("int64_t key = ((int64_t)dist[i] << 32) | (int64_t)i;\n        if (key < best",
                     "int64_t key = ((int64_t)dist[i] << 32) | (int64_t)(nQ - i);\n        if (key < best"),
}


@pytest.fixture(scope="module")
def frames():
    return {1: synth.pinhole_frame_1200()[0], 2: synth.fisheye_frame_1500()[0], 3: synth.clustered_search_20000()[0]}


def _pins(frames):
    tests = [pins.test_hamming_three_routes_agree, pins.test_hamming_special_cases,
             pins.test_sad_window_matches_sliced_bruteforce,
             pins.test_sad_exact_integer_shift_is_zero_at_true_shift,
             pins.test_sad_constant_offset_is_invisible,
             pins.test_subpixel_recovers_vertex_of_exact_parabola,
             pins.test_subpixel_border_and_tie_rules,
             pins.test_predicted_level_matches_log_reading,
             pins.test_kb_projection_matches_generator_and_equidistant_closed_form,
             pins.test_kb_round_trips,
             pins.test_triangulation_exact_on_noise_free_rays_and_equals_lstsq,
             pins.test_fisheye_zero_baseline_rejects_everything]
    for vals, m, keep in [([0, 0, 3], 0, [False] * 3), ([1, 2, 3, 4, 100], 3, [True] * 4 + [False]),
                          ([4, 3, 2, 1], 3, [True] * 4), ([10, 21, 22, 10, 10], 10, [True, False, False, True, True])]:
        tests.append(lambda v=vals, mm=m, k=keep: pins.test_median_keep_hand_lists(v, mm, k))
    for s in (21, 22, 23):
        tests.append(lambda s=s: pins.test_stereo_pinhole_equals_bruteforce(s))
    for s in (31, 32):
        tests.append(lambda s=s: pins.test_fisheye_knn_ratio_equals_bruteforce(s))
    for s in (41, 42, 43):
        tests.append(lambda s=s: pins.test_search_pinhole_equals_bruteforce(s))
    tests.append(lambda: pins.test_search_clustered_equals_bruteforce(51))
    tests.append(pins.test_conflict_hand_built_scene)
    tests.append(pins.test_pinhole_distance_threshold_is_strict)
    tests.append(pins.test_search_ratio_applies_only_to_same_level_second)
    for s in (81, 82):
        tests.append(lambda s=s: pins.test_search_visibility_gates_equal_bruteforce(s))
    tests.append(pins.test_search_visibility_boundaries_are_inclusive)
    tests.append(pins.test_fisheye_parallax_gate_scene)
    tests.append(pins.test_fisheye_depth_gate_scene)
    tests.append(pins.test_fisheye_reprojection_gate_scene)
    tests.append(pins.test_fisheye_needs_two_targets)
    for kind in ("pinhole", "clustered"):
        for d in (0, 1, -1):
            tests.append(lambda k=kind, d=d: motion.test_last_frame_search_equals_bruteforce(k, d))
    for a, c, w in [(10.0, 11.0, 0), (0.0, 174.0, 16), (342.0, 0.0, 29), (11.0, 0.0, 1)]:
        tests.append(lambda a=a, c=c, w=w: motion.test_rotation_bin_closed_forms(a, c, w))
    for cnt, kept in [([5, 9, 9, 1], [0, 1, 2]), ([100, 9, 10, 0], [0, 2]), ([100, 5, 5], [0]),
                      ([3, 3, 3, 3], [0, 1, 2])]:
        tests.append(lambda c=cnt, k=kept: motion.test_three_fullest_rule_closed_forms(c, k))
    for args in [(2, 3, 1, False), (3, 3, 1, True), (4, 3, -1, False), (3, 3, -1, True), (2, 3, 0, True)]:
        tests.append(lambda a=args: motion.test_level_window_follows_the_direction_of_motion(*a))
    tests.append(motion.test_stereo_gate_and_preassigned_flag)
    tests.append(lambda: motion.test_distance_threshold_is_inclusive(100, True))
    tests.append(motion.test_two_points_claiming_one_keypoint)
    for case in mapt.CASES:
        tests.append(lambda c=case: mapt.test_map_update_rule(*c))
    tests.append(mapt.test_random_edit_sequences)
    for args in [([3, 3], 0, 100), ([50], 0, 100)]:
        tests.append(lambda a=args: mapt.test_invalid_edits_are_rejected(*a))
    tests.append(mapt.test_exact_capacity_is_accepted)
    tests.append(pyr.test_level_sizes_of_the_paper_shapes)
    tests.append(lambda: pyr.test_horizontal_ramp_is_round_half_up_of_the_source_column(200, 37))
    tests.append(lambda: pyr.test_vertical_ramp_is_round_half_up_of_the_source_row(40, 250))
    tests.append(pyr.test_exact_halving_is_the_rounded_box_average)
    tests.append(lambda: pyr.test_random_images_match_numpy_resampler(101, 67, 6))
    for bg, fg in [(50, 200), (200, 50)]:
        tests.append(lambda b=bg, f=fg: orb.test_lone_pixel_is_the_only_corner(b, f))
    for t in (7, 20):
        tests.append(lambda t=t: orb.test_threshold_is_strict(t))
    tests.append(lambda: orb.test_scores_are_invariant_under_the_image_symmetries(1))
    tests.append(lambda: orb.test_scores_equal_numpy_brute_force(4, 20, 19))
    tests.append(orb.test_detection_equals_brute_force_on_a_pyramid)
    tests.append(orb.test_plateaus_of_equal_scores_keep_nothing)
    tests.append(orb.test_blur_of_an_impulse_is_the_rounded_binomial_product)
    tests.append(orb.test_blur_keeps_constants_and_interior_ramps_and_clamps_borders)
    for kind, deg in [("+x", 0.0), ("+y", 90.0), ("-x", 180.0), ("+x-y", 315.0)]:
        tests.append(lambda k=kind, d=deg: orb.test_orientation_of_linear_ramps(k, d))
    tests.append(orb.test_orientation_disc_has_radius_15_inclusive)
    for kind in ("+x", "+y", "-x"):
        tests.append(lambda k=kind: orb.test_ramp_descriptors_equal_the_pattern_x_order_in_every_direction(k))
    tests.append(orb.test_diagonal_ramp_descriptor_uses_the_exactly_turned_pattern)
    tests.append(orb.test_descriptors_equal_numpy_brute_force_on_textures)

    def with_frames():
        c1 = (frames[1], oracle.run_frame(frames[1]))
        c2 = (frames[2], oracle.run_frame(frames[2]))
        c3 = (frames[3], oracle.run_frame(frames[3]))
        pins.test_pinhole_stereo_invariants_and_ground_truth(c1)
        pins.test_search_invariants_and_ground_truth(c1, c3)
        pins.test_fisheye_stereo_invariants_and_ground_truth(c2)
        pins.test_fisheye_search_invariants_and_ground_truth(c2)
    tests.append(with_frames)
    return tests


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, frames, tmp_path):
    src = open(os.path.join(HERE, "ft_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new, 1)
    (tmp_path / "ft_oracle.c").write_text(mutated)
    shutil.copy(os.path.join(HERE, "ft_oracle.h"), tmp_path / "ft_oracle.h")
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so, str(tmp_path / "ft_oracle.c"), "-lm"])
    caught = None
    with oracle.using_library(so):
        for t in _pins(frames):
            try:
                t()
            except (AssertionError, TypeError, IndexError, ValueError) as e:
                caught = e
                break
    assert caught is not None, f"no pin caught mutation {name}"
