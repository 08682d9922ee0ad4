"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to an independent fact: a second route to
the same number (numpy unpackbits, a +-1 dot product, a least-squares solver,
a vectorised brute force over all pairs), a closed form (exact integer shifts,
exact parabolas, noise-free triangulation), an invariant, or the generators'
ground truth.  No expected value here comes from the device path.
"""
import numpy as np
import pytest

import oracle
import synth
from synth.fisheye import kb_project64
from tests import brute

f32 = np.float32


# ---------------------------------------------------------------- Hamming ----
def test_hamming_three_routes_agree():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 256, (200, 32), dtype=np.uint8)
    b = rng.integers(0, 256, (200, 32), dtype=np.uint8)
    A, B = brute.bits(a), brute.bits(b)
    by_bits = (A != B).sum(1)
    sa, sb = 2 * A - 1, 2 * B - 1
    by_dot = (256 - (sa * sb).sum(1)) // 2
    ours = np.array([oracle.hamming(a[i], b[i]) for i in range(200)])
    assert (ours == by_bits).all() and (ours == by_dot).all()


def test_hamming_special_cases():
    rng = np.random.default_rng(2)
    a = rng.integers(0, 256, 32, dtype=np.uint8)
    assert oracle.hamming(a, a) == 0
    assert oracle.hamming(a, ~a) == 256
    for bit in (0, 7, 8, 255):
        b = a.copy()
        b[bit // 8] ^= np.uint8(1 << (bit % 8))
        assert oracle.hamming(a, b) == 1


# ------------------------------------------------------------ SAD window ----
def test_sad_window_matches_sliced_bruteforce():
    rng = np.random.default_rng(3)
    for trial in range(60):
        H, W = rng.integers(14, 40), rng.integers(24, 60)
        IL = rng.integers(0, 256, (H, W), dtype=np.uint8)
        IR = rng.integers(0, 256, (H, W), dtype=np.uint8)
        su, sv, su0 = rng.integers(0, W), rng.integers(0, H), rng.integers(0, W)
        want = brute.sad_profile(IL.astype(np.int64), IR.astype(np.int64), su, sv, su0, 5, 5)
        got = oracle.sad_window(IL, IR, int(su), int(sv), int(su0))
        if want is None:
            assert got is None
        else:
            assert got is not None and (got == want).all()


def test_sad_exact_integer_shift_is_zero_at_true_shift():
    rng = np.random.default_rng(4)
    H, W = 40, 80
    IL = rng.integers(0, 256, (H, W), dtype=np.uint8)
    for s in (0, 3, 9):
        IR = np.zeros_like(IL)
        IR[:, :W - s] = IL[:, s:]          # right(x) = left(x + s)
        su, sv = 40, 20
        for k0 in (-3, 0, 2):
            su0 = su - s - k0              # the true shift is k = k0
            sad = oracle.sad_window(IL, IR, su, sv, su0)
            assert sad[k0 + 5] == 0
            assert (sad[np.arange(11) != k0 + 5] > 0).all()


def test_sad_constant_offset_is_invisible():
    """Centre subtraction: adding a constant to the right patch changes nothing."""
    rng = np.random.default_rng(5)
    IL = rng.integers(20, 200, (30, 60), dtype=np.uint8)
    IR = rng.integers(20, 200, (30, 60), dtype=np.uint8)
    a = oracle.sad_window(IL, IR, 30, 15, 28)
    b = oracle.sad_window(IL, (IR.astype(np.int64) + 37).astype(np.uint8), 30, 15, 28)
    assert (a == b).all()


# -------------------------------------------------------------- subpixel ----
def test_subpixel_recovers_vertex_of_exact_parabola():
    rng = np.random.default_rng(6)
    for _ in range(300):
        A = int(rng.integers(1, 200))
        n = int(rng.integers(-A + 1, A))          # x0 = n / (2A), |x0| < 1/2
        kstar = int(rng.integers(-4, 5))
        C = int(rng.integers(0, 1000))
        ks = np.arange(-5, 6)
        d = ks - kstar
        sad = A * d * d - n * d + C              # = A (d - x0)^2 + const
        got = oracle.subpixel(sad)
        assert got is not None
        kb, c, delta = got
        assert kb == kstar and c == C
        assert abs(delta - n / (2 * A)) <= 1e-7


def test_subpixel_border_and_tie_rules():
    assert oracle.subpixel(np.array([0, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14])) is None
    assert oracle.subpixel(np.array([14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 0])) is None
    # two equal minima: the smaller shift wins
    got = oracle.subpixel(np.array([9, 8, 7, 3, 5, 3, 7, 8, 9, 9, 9]))
    assert got[0] == -2
    # |delta| <= 1/2 whatever the three values
    rng = np.random.default_rng(7)
    for _ in range(500):
        s = rng.integers(0, 5000, 11)
        g = oracle.subpixel(s)
        if g is not None:
            assert abs(g[2]) <= 0.5


# ---------------------------------------------------------- median filter ----
@pytest.mark.parametrize("vals,m,keep", [
    ([], -1, []),
    ([5], 5, [True]),
    ([0, 0, 3], 0, [False, False, False]),
    ([1, 2, 3, 4, 100], 3, [True, True, True, True, False]),
    ([4, 3, 2, 1], 3, [True, True, True, True]),
    ([10, 21, 22, 10, 10], 10, [True, False, False, True, True]),
    ([7, 7, 7], 7, [True, True, True]),
])
def test_median_keep_hand_lists(vals, m, keep):
    got_m, got_keep = oracle.median_keep(np.array(vals, np.int32))
    assert got_m == m
    assert list(got_keep) == keep


# -------------------------------------------------------- predicted level ----
def test_predicted_level_matches_log_reading():
    sf = synth.scale_tables()["sf"]
    rng = np.random.default_rng(8)
    ratios = np.exp(rng.uniform(-0.5, 2.3, 4000)).astype(np.float32)
    n_checked = 0
    for r in ratios:
        x = np.log(float(r)) / np.log(1.2)
        if abs(x - round(x)) < 1e-4:
            continue                          # ulp boundary between table and log
        want = int(np.clip(np.ceil(x), 0, 7))
        assert oracle.predict_level(r, sf) == want
        n_checked += 1
    assert n_checked > 3900


# ------------------------------------------------------- Kannala-Brandt ----
def _kb_cam(seed):
    rng = np.random.default_rng(seed)
    return {"fx": f32(190), "fy": f32(190), "cx": f32(256), "cy": f32(256),
            "k": rng.uniform(-0.01, 0.01, 4).astype(np.float32)}


def test_kb_projection_matches_generator_and_equidistant_closed_form():
    cam = _kb_cam(9)
    rng = np.random.default_rng(10)
    X = synth.fisheye.cap_directions(rng, 300, 85.0) * rng.uniform(0.5, 20, 300)[:, None]
    ref = kb_project64(X, cam)
    for i in range(300):
        assert np.abs(oracle.kb_project(cam, X[i]) - ref[i]).max() < 1e-9
    cam0 = dict(cam, k=np.zeros(4, np.float32))
    for i in range(50):
        th = np.arccos(X[i, 2] / np.linalg.norm(X[i]))
        rho = np.hypot(X[i, 0], X[i, 1])
        uv = oracle.kb_project(cam0, X[i])
        assert abs(uv[0] - (256 + 190 * th * X[i, 0] / rho)) < 1e-9
        assert abs(uv[1] - (256 + 190 * th * X[i, 1] / rho)) < 1e-9


def test_kb_round_trips():
    cam = _kb_cam(11)
    rng = np.random.default_rng(12)
    X = synth.fisheye.cap_directions(rng, 300, 80.0) * rng.uniform(0.5, 20, 300)[:, None]
    for i in range(300):
        uv = oracle.kb_project(cam, X[i])
        u32, v32 = f32(uv[0]), f32(uv[1])
        ray = oracle.kb_unproject(cam, u32, v32)
        assert ray is not None
        back = oracle.kb_project(cam, ray)
        assert abs(back[0] - float(u32)) < 1e-9 and abs(back[1] - float(v32)) < 1e-9
        # unproject(project(X)) is parallel to X up to the float32 pixel rounding,
        # where theta_d(theta) is monotone (|k| <= 0.01 keeps it so below 70 deg)
        th = np.arctan2(np.hypot(X[i, 0], X[i, 1]), X[i, 2])
        if th > np.deg2rad(70.0):
            continue
        ray_exact_dir = ray / np.linalg.norm(ray)
        ang = np.arccos(np.clip(ray_exact_dir @ (X[i] / np.linalg.norm(X[i])), -1, 1))
        assert ang < 1e-6
    assert oracle.kb_unproject(cam, f32(256), f32(256))[2] == 1.0
    # beyond the maximal angle the ray is rejected
    assert oracle.kb_unproject(cam, f32(256 + 190 * 1.56), f32(256)) is None


# -------------------------------------------------------- triangulation ----
def test_triangulation_exact_on_noise_free_rays_and_equals_lstsq():
    rng = np.random.default_rng(13)
    R_lr = synth.common.rodrigues(np.array([0.0, 1.0, 0.0]), np.deg2rad(2.0)).astype(np.float32)
    t_lr = np.array([0.1, 0.0, 0.0], np.float32)
    Rd, td = R_lr.astype(np.float64), t_lr.astype(np.float64)
    for _ in range(200):
        X = synth.fisheye.cap_directions(rng, 1, 60.0)[0] * rng.uniform(1, 15)
        Xr = Rd.T @ (X - td)
        r1, r2 = X / X[2], Xr / Xr[2]
        got = oracle.triangulate(r1, r2, R_lr, t_lr)
        assert np.linalg.norm(got - X) <= 1e-9 * np.linalg.norm(X)
        # a different solver on the same linear system
        Rrl, trl = Rd.T, -Rd.T @ td
        A = np.array([[-1, 0, r1[0]], [0, -1, r1[1]],
                      r2[0] * Rrl[2] - Rrl[0], r2[1] * Rrl[2] - Rrl[1]])
        b = np.array([0, 0, -(r2[0] * trl[2] - trl[0]), -(r2[1] * trl[2] - trl[1])])
        ls = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.linalg.norm(got - ls) <= 1e-9 * np.linalg.norm(X)


def test_fisheye_zero_baseline_rejects_everything():
    f = synth.tiny_fisheye(14, n_kp=120)
    f["stereo_cam"]["t_lr"] = np.zeros(3, np.float32)
    f["stereo_cam"]["R_lr"] = np.eye(3, dtype=np.float32)
    # identical images: every ray pair is parallel, so the parallax test rejects
    f["right"] = {k: v.copy() for k, v in f["left"].items()}
    f["stereo_cam"]["right"] = f["stereo_cam"]["left"]
    f["stereo_cam"]["overlap_right"] = f["stereo_cam"]["overlap_left"]
    out = oracle.stereo_fisheye(f)
    assert out["stats"]["ratio_ok"] > 0
    assert out["n_matches"] == 0


# ---------------------------------------------- whole-step brute force ----
@pytest.mark.parametrize("seed", [21, 22, 23, 24, 25])
def test_stereo_pinhole_equals_bruteforce(seed):
    f = synth.tiny_pinhole(seed, n_kp=90)
    got = oracle.stereo_pinhole(f)
    want = brute.stereo_pinhole(f)
    for k in ("right_idx", "dist", "sad"):
        assert (got[k] == want[k]).all(), k
    for k in ("u_right", "depth"):
        assert np.array_equal(got[k].view(np.int32), want[k].astype(np.float32).view(np.int32)), k
    assert got["stats"]["hamming"] == want["stats"]["hamming"]
    assert got["stats"]["median"] == want["stats"]["median"]
    assert got["n_matches"] > 10


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_fisheye_knn_ratio_equals_bruteforce(seed):
    f = synth.tiny_fisheye(seed, n_kp=150)
    H1, j1, H2, ratio_ok = brute.knn2_overlap(f)
    got = oracle.stereo_fisheye(f)
    assert got["stats"]["ratio_ok"] == int(ratio_ok.sum())
    Q = np.nonzero(H1 >= 0)[0]
    assert (got["h2"][Q] == H2[Q]).all()
    m = got["right_idx"] >= 0
    assert ratio_ok[m].all()
    assert (got["right_idx"][m] == j1[m]).all() and (got["dist"][m] == H1[m]).all()


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_search_pinhole_equals_bruteforce(seed):
    f = synth.tiny_pinhole(seed, n_kp=100, n_map=160)
    st = oracle.stereo_pinhole(f)
    for ur in (None, st["u_right"]):
        got = oracle.search_local_points(f, 0, ur)
        want = brute.search_pinhole(f, 0, ur)
        for k in ("mp_match", "mp_dist", "kp_match"):
            assert (got[k] == want[k]).all(), k
        assert got["stats"] == want["stats"]


@pytest.mark.parametrize("seed", [51, 52])
def test_search_clustered_equals_bruteforce(seed):
    f = synth.tiny_clustered(seed)
    got = oracle.search_local_points(f, 0)
    want = brute.search_pinhole(f, 0)
    for k in ("mp_match", "mp_dist", "kp_match"):
        assert (got[k] == want[k]).all(), k
    assert got["n_matches"] > 20


# -------------------------------------------- invariants + ground truth ----
@pytest.fixture(scope="module")
def c1():
    f = synth.pinhole_frame_1200()[0]
    return f, oracle.run_frame(f)


@pytest.fixture(scope="module")
def c2():
    f = synth.fisheye_frame_1500()[0]
    return f, oracle.run_frame(f)


@pytest.fixture(scope="module")
def c3():
    f = synth.clustered_search_20000()[0]
    return f, oracle.run_frame(f)


def _no_duplicates(idx):
    v = idx[idx >= 0]
    return len(np.unique(v)) == len(v)


def test_pinhole_stereo_invariants_and_ground_truth(c1):
    f, r = c1
    st = r["stereo"]
    m = np.nonzero(st["right_idx"] >= 0)[0]
    j = st["right_idx"][m]
    L, R, sf = f["left"], f["right"], f["scales"]["sf"]
    assert _no_duplicates(st["right_idx"])
    assert (np.abs(L["y"][m] - R["y"][j]) <= 2 * sf[R["octave"][j]] + 1).all()
    disp = L["x"][m] - st["u_right"][m]
    maxD = f32(f["stereo_cam"]["bf"]) / f32(f["stereo_cam"]["b"])
    assert (disp >= 0).all() and (disp < maxD).all()
    assert (np.abs(L["octave"][m].astype(int) - R["octave"][j].astype(int)) <= 1).all()
    assert (st["dist"][m] < 75).all()
    assert (st["dist"][m] == brute.hamming_matrix(L["desc"][m], R["desc"])[np.arange(len(m)), j]).all()
    rel = np.abs(st["depth"][m].astype(np.float64) * disp - float(f["stereo_cam"]["bf"]))
    assert (rel <= 2e-7 * float(f["stereo_cam"]["bf"])).all()
    truth = dict(map(tuple, f["truth"]["stereo_pairs"].tolist()))
    good = sum(truth.get(int(i)) == int(st["right_idx"][i]) for i in m)
    assert good >= 0.97 * len(m) and good >= 0.75 * len(truth)
    # sub-pixel disparity tracks the generating disparity field
    d_true = {int(i): f["truth"]["disparity"][k] for k, i in enumerate(f["truth"]["stereo_pairs"][:, 0])}
    err = [disp[q] - d_true[int(i)] for q, i in enumerate(m) if truth.get(int(i)) == int(st["right_idx"][i])]
    assert np.median(np.abs(err)) < 0.3


def _check_search(f, s, view, u_right=None):
    spec = f["search"][view]
    kp = f[spec["image"]]
    assert _no_duplicates(s["mp_match"])
    m = np.nonzero(s["mp_match"] >= 0)[0]
    k = s["mp_match"][m]
    assert (s["kp_match"][k] == m).all()
    assert (s["kp_match"] >= 0).sum() == len(m)
    assert (s["mp_dist"][m] <= 100).all()
    assert (s["mp_dist"][m] == brute.hamming_matrix(f["map"]["desc"][m], kp["desc"])[np.arange(len(m)), k]).all()
    if spec.get("preassigned") is not None:
        assert not spec["preassigned"][k].any()


def test_search_invariants_and_ground_truth(c1, c3):
    for f, r in (c1, c3):
        s = r["search"][0]
        _check_search(f, s, 0)
        truth = dict(map(tuple, f["truth"]["map_kp"].tolist()))
        m = np.nonzero(s["mp_match"] >= 0)[0]
        good = sum(truth.get(int(i)) == int(s["mp_match"][i]) for i in m)
        assert good >= 0.97 * len(m)
        assert good >= 0.6 * len(truth)


def test_pinhole_projection_round_trip(c3):
    f, _ = c3
    cam = f["search"][0]["cam"]
    P = f["map"]["pos"][:500]
    Pc = (cam["R"].astype(np.float64) @ P.T.astype(np.float64)).T + cam["t"]
    u = float(cam["fx"]) * Pc[:, 0] / Pc[:, 2] + float(cam["cx"])
    v = float(cam["fy"]) * Pc[:, 1] / Pc[:, 2] + float(cam["cy"])
    back = np.stack([(u - float(cam["cx"])) * Pc[:, 2] / float(cam["fx"]),
                     (v - float(cam["cy"])) * Pc[:, 2] / float(cam["fy"]), Pc[:, 2]], 1)
    assert np.abs(back - Pc).max() <= 1e-6 * np.abs(Pc).max()
    # the camera centre supplied with the pose is -R^T t
    O = -cam["R"].astype(np.float64).T @ cam["t"].astype(np.float64)
    assert np.abs(O - cam["O"]).max() < 1e-6


def test_fisheye_stereo_invariants_and_ground_truth(c2):
    f, r = c2
    st = r["stereo"]
    assert _no_duplicates(st["right_idx"])
    m = np.nonzero(st["right_idx"] >= 0)[0]
    assert len(m) > 50
    j = st["right_idx"][m]
    H1, j1, H2, ratio_ok = brute.knn2_overlap(f)
    assert ratio_ok[m].all() and (j1[m] == j).all()
    assert (st["depth"][m] > 0).all()
    truth = dict(map(tuple, f["truth"]["stereo_pairs"].tolist()))
    good = sum(truth.get(int(i)) == int(st["right_idx"][i]) for i in m)
    assert good >= 0.97 * len(m)
    # triangulated points reproject onto both keypoints (generator's projector)
    cam = f["stereo_cam"]
    X = st["xyz"][m].astype(np.float64)
    uvL = kb_project64(X, cam["left"])
    Rl, tl = cam["R_lr"].astype(np.float64), cam["t_lr"].astype(np.float64)
    uvR = kb_project64((X - tl) @ Rl, cam["right"])
    s2 = f["scales"]["sigma2"]
    eL = ((uvL - np.stack([f["left"]["x"][m], f["left"]["y"][m]], 1)) ** 2).sum(1)
    eR = ((uvR - np.stack([f["right"]["x"][j], f["right"]["y"][j]], 1)) ** 2).sum(1)
    assert (eL <= 5.991 * s2[f["left"]["octave"][m]] * (1 + 1e-5)).all()
    assert (eR <= 5.991 * s2[f["right"]["octave"][j]] * (1 + 1e-5)).all()


def test_fisheye_search_invariants_and_ground_truth(c2):
    f, r = c2
    for v in range(2):
        _check_search(f, r["search"][v], v)
        assert r["search"][v]["n_matches"] > 300


def test_conflict_hand_built_scene():
    """Two map points whose projections fall on the same keypoint with the same
    descriptor distance: the smaller map-point index keeps it; with distances
    4 and 2 the closer one keeps it, whatever its index."""
    f = synth.tiny_pinhole(61, n_kp=40, n_map=4)
    kp = f["left"]
    cam = f["search"][0]["cam"]
    cam["R"] = np.eye(3, dtype=np.float32); cam["t"] = np.zeros(3, np.float32)
    cam["O"] = np.zeros(3, np.float32)
    f["search"][0]["preassigned"][:] = 0
    k = 7
    Z = 5.0
    P = np.array([(float(kp["x"][k]) - float(cam["cx"])) * Z / float(cam["fx"]),
                  (float(kp["y"][k]) - float(cam["cy"])) * Z / float(cam["fy"]), Z])
    mp = f["map"]
    lvl = int(kp["octave"][k])
    for m in range(4):
        mp["pos"][m] = P + np.array([1e-4 * m, 0, 0])
        mp["normal"][m] = P / np.linalg.norm(P)
        mp["dmax"][m] = np.float32(np.linalg.norm(P) * float(f["scales"]["sf"][lvl]))
        mp["dmin"][m] = np.float32(mp["dmax"][m] / float(f["scales"]["sf"][7]))
        mp["desc"][m] = kp["desc"][k]
    far = np.float32(1e6)
    kp["x"][np.arange(len(kp["x"])) != k] = far    # leave a single candidate
    flips = [4, 4, 2, 6]
    for m in range(4):
        d = mp["desc"][m].copy()
        for b in range(flips[m]):
            d[b] ^= 1
        mp["desc"][m] = d
    out = oracle.search_local_points(f, 0)
    assert out["mp_match"].tolist() == [-1, -1, k, -1]
    assert out["kp_match"][k] == 2
    flips = [4, 4, 5, 6]
    for m in range(4):
        d = kp["desc"][k].copy()
        for b in range(flips[m]):
            d[b] ^= 1
        mp["desc"][m] = d
    out = oracle.search_local_points(f, 0)
    assert out["mp_match"].tolist() == [k, -1, -1, -1]


def _stereo_pair_with_distance(seed, flips):
    """A tiny pinhole frame whose first matched pair gets its right descriptor
    replaced by the left one with exactly `flips` bits flipped."""
    f = synth.tiny_pinhole(seed, n_kp=60)
    base = oracle.stereo_pinhole(f)
    i = int(np.nonzero(base["right_idx"] >= 0)[0][0])
    j = int(base["right_idx"][i])
    d = f["left"]["desc"][i].copy()
    bitsd = np.unpackbits(d, bitorder="little")
    bitsd[:flips] ^= 1
    f["right"]["desc"][j] = np.packbits(bitsd, bitorder="little")
    return f, i, j


def test_pinhole_distance_threshold_is_strict():
    f, i, j = _stereo_pair_with_distance(71, 74)
    out = oracle.stereo_pinhole(f)
    assert out["right_idx"][i] == j and out["dist"][i] == 74
    f, i, j = _stereo_pair_with_distance(71, 75)
    out = oracle.stereo_pinhole(f)
    assert out["right_idx"][i] != j


def test_search_ratio_applies_only_to_same_level_second():
    """One map point, two candidates at distances 20 and 22: same level -> the
    ratio test (5*20 > 4*22) rejects; different levels -> accepted."""
    f = synth.tiny_pinhole(62, n_kp=40, n_map=1)
    kp, mp = f["left"], f["map"]
    cam = f["search"][0]["cam"]
    cam["R"] = np.eye(3, dtype=np.float32); cam["t"] = np.zeros(3, np.float32)
    cam["O"] = np.zeros(3, np.float32)
    f["search"][0]["preassigned"][:] = 0
    a, b = 5, 9
    kp["x"][:] = np.float32(1e6)
    kp["x"][a] = np.float32(100.0); kp["y"][a] = np.float32(60.0)
    kp["x"][b] = np.float32(101.0); kp["y"][b] = np.float32(61.0)
    Z = 5.0
    P = np.array([(100.0 - float(cam["cx"])) * Z / float(cam["fx"]),
                  (60.0 - float(cam["cy"])) * Z / float(cam["fy"]), Z])
    mp["pos"][0] = P
    mp["normal"][0] = P / np.linalg.norm(P)
    mp["dmax"][0] = np.float32(np.linalg.norm(P) * float(f["scales"]["sf"][2]))
    mp["dmin"][0] = np.float32(mp["dmax"][0] / float(f["scales"]["sf"][7]))
    base = mp["desc"][0]
    for k, n in ((a, 20), (b, 22)):
        bb = np.unpackbits(base.copy(), bitorder="little")
        bb[:n] ^= 1
        kp["desc"][k] = np.packbits(bb, bitorder="little")
    kp["octave"][a] = 2; kp["octave"][b] = 2
    out = oracle.search_local_points(f, 0)
    assert out["mp_match"][0] == -1
    kp["octave"][b] = 3
    out = oracle.search_local_points(f, 0)
    assert out["mp_match"][0] == a and out["mp_dist"][0] == 20
    # the second found first in index order (b < a) must still count
    kp["octave"][b] = 2
    kp["desc"][a], kp["desc"][b] = kp["desc"][b].copy(), kp["desc"][a].copy()
    out = oracle.search_local_points(f, 0)
    assert out["mp_match"][0] == -1


# ------------------------------------------- visibility tests of the search ----
def _gate_frames(seed):
    from synth.gates import add_gate_cases
    out = []
    for base in (synth.tiny_pinhole(seed, n_kp=100, n_map=220), synth.tiny_clustered(seed)):
        g, cases = add_gate_cases(base, seed, frac=0.06, n_edge=6)
        out.append((g, cases))
    return out


@pytest.mark.parametrize("seed", [81, 82])
def test_search_visibility_gates_equal_bruteforce(seed):
    """Map points seen too near, too far and from the side, and points on the
    exact binary32 boundary of each test: the oracle's per-test rejection
    counts and matches equal the all-pairs brute force, and each test rejects
    its own cases."""
    from synth.gates import gate_outcomes
    for g, cases in _gate_frames(seed):
        edge = gate_outcomes(g, cases)
        for name, ok in edge.items():
            assert ok.all() if name.endswith("_in") else not ok.any(), name
        st = oracle.stereo_pinhole(g) if g["kind"] == "pinhole" else None
        for ur in ((None, st["u_right"]) if st else (None,)):
            got = oracle.search_local_points(g, 0, ur)
            want = brute.search_pinhole(g, 0, ur)
            assert got["stats"] == want["stats"]
            for k in ("mp_match", "mp_dist", "kp_match"):
                assert (got[k] == want[k]).all(), k
            s = got["stats"]
            # every far-off case is rejected by its own test (some may already
            # fall outside the image); edge cases outside their bound too
            for name, key in (("near", "rej_near"), ("far", "rej_far"), ("angle", "rej_angle")):
                assert s[key] >= len(cases[name]) + len(cases[name + "_out"]) - s["rej_frame"]
                assert s[key] > 0


def test_search_visibility_boundaries_are_inclusive():
    """A map point whose distance equals dist_lo*dmin or dist_hi*dmax exactly,
    or whose viewing cosine equals the limit exactly, is visible; one binary32
    step beyond is not (the tests are >= / <= / >=)."""
    f = synth.tiny_pinhole(83, n_kp=60, n_map=1)
    cam = f["search"][0]["cam"]
    cam["R"] = np.eye(3, dtype=np.float32); cam["t"] = np.zeros(3, np.float32)
    cam["O"] = np.zeros(3, np.float32)
    mp = f["map"]
    P = np.array([0.5, -0.25, 4.0], np.float32)
    mp["pos"][0] = P
    dist = np.sqrt((P[0] * P[0] + P[1] * P[1]) + P[2] * P[2]).astype(np.float32)
    ray = P.astype(np.float64) / np.linalg.norm(P.astype(np.float64))
    mp["normal"][0] = ray.astype(np.float32)
    sp = f["search_params"]
    from synth.gates import _first_passing_max, _last_passing_min

    def visible():
        return oracle.search_local_points(f, 0)["stats"]["visible"] == 1
    mp["dmax"][0] = np.float32(dist * 2); mp["dmin"][0] = np.float32(dist / 2)
    assert visible()
    d = _last_passing_min(dist, np.float32(sp["dist_lo"]))
    mp["dmin"][0] = d
    if np.float32(np.float32(sp["dist_lo"]) * d) == dist:
        assert visible()
    mp["dmin"][0] = np.nextafter(d, np.float32(np.inf))
    assert not visible()
    mp["dmin"][0] = np.float32(dist / 2)
    d = _first_passing_max(dist, np.float32(sp["dist_hi"]))
    mp["dmax"][0] = d
    assert visible()
    mp["dmax"][0] = np.nextafter(d, np.float32(0))
    assert not visible()


# ------------------------------------- triangulation check of fisheye pairs ----
def _scene_check(f, reasons_needed):
    from tests import fisheye_scenes as fs
    exp = fs.expected(f)
    out = oracle.stereo_fisheye(f)
    got = out["right_idx"] == np.arange(len(exp))
    n_clear = 0
    for i, (acc, reason, clear) in enumerate(exp):
        if clear:
            n_clear += 1
            assert got[i] == acc, (i, reason)
    seen = {}
    for acc, reason, clear in exp:
        if clear:
            seen[reason] = seen.get(reason, 0) + 1
    for r in reasons_needed:
        assert seen.get(r, 0) >= 3, (r, seen)
    return exp, out


def test_fisheye_parallax_gate_scene():
    """Noise-free pairs with parallax cosines just below and just above the
    limit: accepted below, rejected above (the depth and reprojection tests
    pass for all of them)."""
    from tests import fisheye_scenes as fs
    f = fs.parallax_scene()
    _, out = _scene_check(f, ["ok", "parallax"])
    assert out["stats"]["rej_parallax"] >= 3


def test_fisheye_depth_gate_scene():
    """Lines that meet behind one camera and in front of the other are
    rejected by the depth test of that camera, with the reprojection gate
    opened so that nothing else could reject them."""
    from tests import fisheye_scenes as fs
    f = fs.depth_scene()
    exp, out = _scene_check(f, ["ok", "depth"])
    L = f["left"]
    # both halves are present: behind the right camera and behind the left one
    cam = f["stereo_cam"]
    R, t = cam["R_lr"].astype(np.float64), cam["t_lr"].astype(np.float64)
    behind = {"left": 0, "right": 0}
    for i, (acc, reason, clear) in enumerate(exp):
        if reason != "depth":
            continue
        r1 = fs.unproject(cam["left"], L["x"][i], L["y"][i])
        r2 = fs.unproject(cam["right"], f["right"]["x"][i], f["right"]["y"][i])
        X = fs.lstsq_point(r1, r2, R, t)
        behind["left" if X[2] <= 0 else "right"] += 1
    assert behind["left"] >= 3 and behind["right"] >= 3
    assert out["stats"]["rej_depth"] == sum(e[1] == "depth" for e in exp)


def test_fisheye_reprojection_gate_scene():
    """Right keypoints moved off the exact projection, with the two keypoints
    on levels whose gates differ 12.8x: each view is judged against its own
    keypoint's level.  The scene holds pairs that only the right view's own
    level rejects, pairs that pass only with the full chi2 bound (not half),
    and the same two kinds for the left view."""
    from tests import fisheye_scenes as fs
    f = fs.reprojection_scene()
    exp, _ = _scene_check(f, ["ok", "reproj"])
    cam, sc, sp = f["stereo_cam"], f["scales"], f["stereo_params"]
    L, Rk = f["left"], f["right"]
    R, t = cam["R_lr"].astype(np.float64), cam["t_lr"].astype(np.float64)
    s2 = sc["sigma2"].astype(np.float64)
    kinds = {"right_own_level": 0, "right_full_bound": 0, "left_own_level": 0, "left_full_bound": 0}
    for i, (acc, reason, clear) in enumerate(exp):
        if not clear or reason not in ("ok", "reproj"):
            continue
        r1 = fs.unproject(cam["left"], L["x"][i], L["y"][i])
        r2 = fs.unproject(cam["right"], Rk["x"][i], Rk["y"][i])
        X = fs.lstsq_point(r1, r2, R, t)
        eL = ((kb_project64(X[None], cam["left"])[0] - [L["x"][i], L["y"][i]]) ** 2).sum()
        eR = ((kb_project64((R.T @ (X - t))[None], cam["right"])[0] - [Rk["x"][i], Rk["y"][i]]) ** 2).sum()
        oL, oR = int(L["octave"][i]), int(Rk["octave"][i])
        gL, gR = sp["chi2"] * s2[oL], sp["chi2"] * s2[oR]
        if eL <= gL and gR < eR <= sp["chi2"] * s2[oL]:
            kinds["right_own_level"] += 1
        if eL <= gL and 0.5 * gR < eR <= gR:
            kinds["right_full_bound"] += 1
        if eR <= gR and gL < eL <= sp["chi2"] * s2[oR]:
            kinds["left_own_level"] += 1
        if eR <= gR and 0.5 * gL < eL <= gL:
            kinds["left_full_bound"] += 1
    assert all(v >= 2 for v in kinds.values()), kinds


def test_fisheye_needs_two_targets():
    """With one right keypoint in the overlap there is no second nearest
    distance, so nothing is matched; a second target makes matches possible."""
    from tests import fisheye_scenes as fs
    f = fs.parallax_scene()
    ok = [i for i, e in enumerate(fs.expected(f)) if e[0] and e[2]]
    i = ok[0]
    W = f["size"]["W"]
    xr = f["right"]["x"][i]
    f["stereo_cam"]["overlap_right"] = np.array([xr, xr], np.float32)
    others = np.nonzero(f["right"]["x"] == xr)[0]
    assert len(others) == 1
    out = oracle.stereo_fisheye(f)
    assert out["stats"]["T"] == 1 and out["n_matches"] == 0
    j = ok[1]
    f["right"]["x"][j] = xr
    out = oracle.stereo_fisheye(f)
    assert out["stats"]["T"] == 2 and out["right_idx"][i] == i
    f["stereo_cam"]["overlap_right"] = np.array([0, W], np.float32)
