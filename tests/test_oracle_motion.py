"""Pins of the oracle's last-frame search by projection (Section II-C, Initial
Pose Estimation: the previous frame's map points are projected into the
current frame and matched against its features; Section IV-E: the same
search-by-projection kernel serves this call site).

Expected values come from an independent numpy brute force over every
(point, keypoint) pair, from hand-built scenes whose outcome follows from the
definition, from closed forms of the rotation bin and the three-fullest rule,
and from the generator's ground truth.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import brute

f32 = np.float32


def _frames():
    return {"pinhole": synth.tiny_pinhole(901), "clustered": synth.tiny_clustered(902)}


def _equal(a, b):
    for k in ("last_match", "last_dist", "kp_match"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert a["kept_bins"] == b["kept_bins"]


@pytest.mark.parametrize("direction", [0, 1, -1])
@pytest.mark.parametrize("kind", ["pinhole", "clustered"])
def test_last_frame_search_equals_bruteforce(kind, direction):
    f = _frames()[kind]
    for seed in (1, 2):
        case = synth.last_frame_case(f, 910 + seed, direction=direction)
        got = oracle.search_last_frame(case)
        want = brute.search_last_frame_pinhole(case)
        _equal(got, want)
        for k in ("in_image", "candidates", "accepted", "matches"):
            assert got["stats"][k] == want["stats"][k], k


def test_last_frame_search_full_size_equals_bruteforce():
    """The 1200-keypoint pinhole frame with its stereo right coordinates, and
    the clustered scene (3000 keypoints), without the rotation check too."""
    for f, seed in ((synth.pinhole_frame_1200()[0], 921), (synth.clustered_search_20000()[0], 922)):
        for rot in (1, 0):
            case = synth.last_frame_case(f, seed, check_orientation=rot)
            got = oracle.search_last_frame(case)
            _equal(got, brute.search_last_frame_pinhole(case))
            assert got["n_matches"] > 100


@pytest.mark.parametrize("a_last,a_cur,want", [
    (0.0, 0.0, 0), (10.0, 10.0, 0), (10.0, 11.0, 0),     # -1 deg -> 359 -> 29.92 -> 30 -> wraps to 0
    (180.0, 0.0, 15), (11.0, 0.0, 1), (17.0, 0.0, 1), (19.0, 0.0, 2),
    (0.0, 174.0, 16), (359.0, 0.0, 0), (353.0, 0.0, 29), (342.0, 0.0, 29),
    (400.0, 0.0, 3), (0.0, 500.0, 18), (720.0, 0.0, 0)])   # angles outside [0, 360): bin modulo 30
def test_rotation_bin_closed_forms(a_last, a_cur, want):
    """30 bins of 12 degrees centred on multiples of 12: a rotation r lands in
    bin round(r / 12) mod 30 (after adding 360 to a negative rotation)."""
    assert oracle.rotation_bin(a_last, a_cur, 30) == want
    assert brute.rotation_bins([a_last], [a_cur], 30)[0] == want


@pytest.mark.parametrize("count,kept", [
    ([5, 9, 9, 1], [0, 1, 2]),           # ties: the lower bin ranks first
    ([100, 9, 10, 0], [0, 2]),           # 10 * 10 >= 100 keeps bin 2; 10 * 9 < 100 drops bin 1
    ([100, 5, 5], [0]),                  # second below a tenth: second and third dropped
    ([0, 0, 7], [2]),
    ([3, 3, 3, 3], [0, 1, 2]),
    ([0, 0, 0], []),
    ([1, 0, 0, 40, 4, 4], [3, 4, 5])])
def test_three_fullest_rule_closed_forms(count, kept):
    got = oracle.three_fullest(count)
    assert sorted(np.nonzero(got)[0].tolist()) == kept
    assert sorted(np.nonzero(brute.three_fullest(count))[0].tolist()) == kept


def _scene(k_oct, lo, direction, ka=10.0, la=10.0, ur=None, pre=None):
    """One last point projecting exactly onto keypoint 0 at (100, 80), one
    distractor keypoint far away; identity pose, fx = 100, centre (100, 80)."""
    sc = synth.scale_tables()
    d = np.random.default_rng(0).integers(0, 256, (2, 32), dtype=np.uint8)
    kps = {"x": np.array([100.0, 10.0], f32), "y": np.array([80.0, 10.0], f32),
           "octave": np.array([k_oct, 0], np.uint8), "desc": d, "angle": np.array([ka, 0.0], f32)}
    cam = {"model": 0, "fx": f32(100), "fy": f32(100), "cx": f32(100), "cy": f32(80),
           "k": np.zeros(4, f32), "bf": f32(10.0), "bounds": np.array([0, 200, 0, 160], f32),
           "R": np.eye(3, dtype=f32), "t": np.zeros(3, f32), "O": np.zeros(3, f32)}
    return {"kind": "last_frame", "scales": sc,
            "last": {"pos": np.array([[0.0, 0.0, 2.0]], f32), "desc": d[:1].copy(),
                     "octave": np.array([lo], np.uint8), "angle": np.array([la], f32)},
            "kps": kps, "cam": cam, "grid": (8, 8), "preassigned": pre, "u_right": ur,
            "params": synth.motion_params(direction=direction)}


@pytest.mark.parametrize("k_oct,lo,direction,found", [
    (3, 3, 0, True), (2, 3, 0, True), (4, 3, 0, True), (1, 3, 0, False), (5, 3, 0, False),
    (3, 3, 1, True), (7, 3, 1, True), (2, 3, 1, False),
    (3, 3, -1, True), (0, 3, -1, True), (4, 3, -1, False)])
def test_level_window_follows_the_direction_of_motion(k_oct, lo, direction, found):
    r = oracle.search_last_frame(_scene(k_oct, lo, direction))
    assert (r["last_match"][0] == 0) == found
    assert r["n_matches"] == int(found)


def test_stereo_gate_and_preassigned_flag():
    """The projected right coordinate of the point is 100 - 10 / 2 = 95; the
    radius at octave 0 is 7."""
    for ur, found in ((95.0, True), (101.9, True), (102.1, False), (-1.0, True), (0.0, True)):
        case = _scene(0, 0, 0, ur=np.array([ur, -1.0], f32))
        assert (oracle.search_last_frame(case)["last_match"][0] == 0) == found, ur
    case = _scene(0, 0, 0, pre=np.array([1, 0], np.uint8))
    assert oracle.search_last_frame(case)["last_match"][0] == -1


def test_generator_ground_truth_is_mostly_recovered():
    """Diagnostic against the generator's known pairs (not parity): most true
    points find their keypoint; accepted matches are within the distance
    threshold; no keypoint is matched twice; the kept bins hold the frame's
    5-degree image rotation."""
    for gen, seed in ((synth.pinhole_frame_1200, 931), (synth.fisheye_frame_1500, 932)):
        f = gen()[0]
        case = synth.last_frame_case(f, seed)
        r = oracle.search_last_frame(case)
        tr = case["truth"]["last_kp"]
        assert (r["last_match"][tr[:, 0]] == tr[:, 1]).mean() > 0.6
        m = r["last_match"] >= 0
        assert (r["last_dist"][m] <= 100).all()
        assert len(np.unique(r["last_match"][m])) == m.sum()
        assert 0 in r["kept_bins"]
        assert r["stats"]["matches"] < r["stats"]["after_conflict"]   # the rotation check dropped some


def _flip(d, n):
    """d with its first n bits flipped (distance exactly n)."""
    bits = np.unpackbits(d, bitorder="little")
    bits[:n] ^= 1
    return np.packbits(bits, bitorder="little")


@pytest.mark.parametrize("dist,found", [(0, True), (99, True), (100, True), (101, False), (180, False)])
def test_distance_threshold_is_inclusive(dist, found):
    case = _scene(0, 0, 0)
    case["last"]["desc"] = _flip(case["kps"]["desc"][0].copy(), dist)[None, :]
    r = oracle.search_last_frame(case)
    assert (r["last_match"][0] == 0) == found
    if found:
        assert r["last_dist"][0] == dist


def test_two_points_claiming_one_keypoint():
    """Two last points project onto keypoint 0: the one at the smaller distance
    keeps it; at equal distances the smaller point index keeps it; the loser is
    unmatched (no second choice)."""
    for d0, d1, winner in ((30, 20, 1), (20, 30, 0), (25, 25, 0)):
        case = _scene(0, 0, 0)
        k0 = case["kps"]["desc"][0]
        case["last"] = {"pos": np.array([[0.0, 0.0, 2.0], [0.0, 0.0, 4.0]], f32),
                        "desc": np.stack([_flip(k0.copy(), d0), _flip(k0.copy(), d1)]),
                        "octave": np.array([0, 0], np.uint8), "angle": np.array([10.0, 10.0], f32)}
        r = oracle.search_last_frame(case)
        assert r["last_match"][winner] == 0 and r["last_match"][1 - winner] == -1
        assert r["kp_match"][0] == winner
        assert r["stats"]["accepted"] == 2 and r["stats"]["after_conflict"] == 1
