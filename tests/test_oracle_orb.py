"""Pins of the oracle's ORB extraction (keypoints on every pyramid level and
their descriptors: Section II-A, Section IV-B).

The paper fixes none of the detector's details; the readings (FAST-9 score,
strict 3x3 non-maximum suppression, intensity-centroid orientation over a
radius-15 disc, binomial smoothing, a caller-supplied point-pair pattern
turned exactly by the centroid angle) are pinned by closed forms on
hand-built images, by symmetries any mistake in the ring or the signs
breaks, and by a numpy brute force written independently of the C code.
"""
import math

import numpy as np
import pytest

import oracle
import synth

RING = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
        (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]
BINOM = np.array([1, 6, 15, 20, 15, 6, 1], np.int64)


def texture(seed, h=96, w=128):
    """Smooth random texture with strong local contrast (many corners)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 1, (h + 8, w + 8))
    k = np.exp(-0.5 * (np.arange(-4, 5) / 1.3) ** 2)
    a = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 1, a)
    a = np.apply_along_axis(lambda c: np.convolve(c, k, "same"), 0, a)[4:-4, 4:-4]
    a = (a - a.mean()) / a.std()
    return np.clip(128 + 50 * a, 0, 255).astype(np.uint8)


def brute_scores(img, t, edge):
    """FAST-9 scores by numpy: shifted copies of the image for the 16 ring
    offsets, the arc minimum by a sliding window over the ring."""
    img = img.astype(np.int32)
    H, W = img.shape
    out = np.zeros((H, W), np.int32)
    ys, xs = slice(edge, H - edge), slice(edge, W - edge)
    c = img[ys, xs]
    ring = np.stack([img[edge + dy:H - edge + dy, edge + dx:W - edge + dx] for dx, dy in RING])
    best = np.full(c.shape, -1, np.int32)
    for sign in (1, -1):
        d = sign * (ring - c[None])
        d2 = np.concatenate([d, d[:8]])                 # arcs wrap around the ring
        for a in range(16):
            best = np.maximum(best, d2[a:a + 9].min(axis=0) - 1)
    out[ys, xs] = np.where(best >= t, best, 0)
    return out


def brute_nms(s):
    H, W = s.shape
    p = np.pad(s, 1)
    keep = s > 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                keep &= s > p[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    return keep


def single_level(img):
    h, w = img.shape
    return {"data": img.reshape(-1).copy(), "offset": np.array([0], np.int64),
            "width": np.array([w], np.int32), "height": np.array([h], np.int32)}


# ---------------------------------------------------------------- FAST score
@pytest.mark.parametrize("bg,fg", [(50, 200), (200, 50), (0, 255)])
def test_lone_pixel_is_the_only_corner(bg, fg):
    img = np.full((64, 64), bg, np.uint8)
    img[30, 33] = fg
    s = oracle.fast_score_map(img, 20, 19)
    assert np.argwhere(s).tolist() == [[30, 33]]
    assert s[30, 33] == abs(fg - bg) - 1


@pytest.mark.parametrize("t", [1, 7, 20, 60])
def test_threshold_is_strict(t):
    img = np.full((48, 48), 100, np.uint8)
    img[24, 24] = 100 + t                               # every ring pixel exactly t darker
    assert oracle.fast_score_map(img, t, 19).max() == 0
    img[24, 24] = 100 + t + 1
    s = oracle.fast_score_map(img, t, 19)
    assert s[24, 24] == t and np.count_nonzero(s) == 1


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("at", [20, 27, 31])
def test_straight_step_edges_have_no_corners(axis, at):
    img = np.full((60, 60), 40, np.uint8)
    if axis == 0:
        img[at:, :] = 220
    else:
        img[:, at:] = 220
    assert oracle.fast_score_map(img, 10, 19).max() == 0


def test_constant_and_gentle_ramps_have_no_corners():
    assert oracle.fast_score_map(np.full((50, 50), 77, np.uint8), 1, 19).max() == 0
    y, x = np.mgrid[0:50, 0:50]
    ramp = (20 + 6 * x // 2 + 3 * y // 2).astype(np.uint8)   # ring differences stay below 21
    assert oracle.fast_score_map(ramp, 20, 19).max() == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_scores_are_invariant_under_the_image_symmetries(seed):
    img = texture(seed)
    t = 12
    s = oracle.fast_score_map(img, t, 19)
    assert np.count_nonzero(s) > 50
    lo, hi = int(img.min()), int(img.max())
    if hi + 5 <= 255:
        assert np.array_equal(oracle.fast_score_map(img + np.uint8(5), t, 19), s)
    if lo >= 5:
        assert np.array_equal(oracle.fast_score_map(img - np.uint8(5), t, 19), s)
    assert np.array_equal(oracle.fast_score_map(255 - img, t, 19), s)
    sq = img[:, :96]
    ss = oracle.fast_score_map(sq, t, 19)
    assert np.array_equal(oracle.fast_score_map(np.ascontiguousarray(sq.T), t, 19), ss.T)
    assert np.array_equal(oracle.fast_score_map(np.ascontiguousarray(img[::-1, ::-1]), t, 19), s[::-1, ::-1])
    assert np.array_equal(oracle.fast_score_map(np.ascontiguousarray(img[:, ::-1]), t, 19), s[:, ::-1])


@pytest.mark.parametrize("seed,t,edge", [(4, 20, 19), (5, 7, 19), (6, 35, 22)])
def test_scores_equal_numpy_brute_force(seed, t, edge):
    img = texture(seed)
    assert np.array_equal(oracle.fast_score_map(img, t, edge), brute_scores(img, t, edge))


# ------------------------------------------------------------------ detection
def test_detection_equals_brute_force_on_a_pyramid():
    sc = synth.scale_tables()
    img = texture(7, 240, 320)
    pyr = oracle.pyramid(img, sc["inv_sf"])
    got = oracle.orb_detect(pyr, sc["sf"], t=15, edge=19)
    want = {k: [] for k in ("lx", "ly", "octave", "score")}
    for l in range(8):
        w, h, o = int(pyr["width"][l]), int(pyr["height"][l]), int(pyr["offset"][l])
        lvl = pyr["data"][o:o + w * h].reshape(h, w)
        s = brute_scores(lvl, 15, 19)
        ys, xs = np.nonzero(brute_nms(s))                 # row-major: (y, x) order
        want["lx"] += xs.tolist(); want["ly"] += ys.tolist()
        want["octave"] += [l] * len(xs); want["score"] += s[ys, xs].tolist()
    assert got["count"] == len(want["lx"]) > 100
    for k in want:
        assert got[k].tolist() == want[k], k
    sf = sc["sf"].astype(np.float32)
    assert np.array_equal(got["x"], got["lx"].astype(np.float32) * sf[got["octave"]])
    assert np.array_equal(got["y"], got["ly"].astype(np.float32) * sf[got["octave"]])
    assert (got["lx"] >= 19).all() and (got["ly"] >= 19).all()
    assert (got["lx"] < pyr["width"][got["octave"]] - 19).all()
    assert (got["ly"] < pyr["height"][got["octave"]] - 19).all()


def test_plateaus_of_equal_scores_keep_nothing():
    img = np.full((64, 64), 50, np.uint8)
    img[30, 30] = img[30, 31] = 200                     # two adjacent equal corners
    s = oracle.fast_score_map(img, 20, 19)
    assert s[30, 30] == s[30, 31] > 0
    got = oracle.orb_detect(single_level(img), np.ones(1, np.float32), t=20, edge=19)
    assert got["count"] == 0
    img[30, 31] = 199                                   # now one is higher
    got = oracle.orb_detect(single_level(img), np.ones(1, np.float32), t=20, edge=19)
    assert got["count"] == 1 and (got["lx"][0], got["ly"][0]) == (30, 30)


def test_capacity_keeps_the_first_in_order_and_reports_the_count():
    sc = synth.scale_tables()
    pyr = oracle.pyramid(texture(8, 200, 260), sc["inv_sf"])
    full = oracle.orb_detect(pyr, sc["sf"], t=12, edge=19)
    part = oracle.orb_detect(pyr, sc["sf"], t=12, edge=19, cap=full["count"] // 3)
    assert part["count"] == full["count"]
    k = full["count"] // 3
    for key in ("lx", "ly", "octave", "score", "x", "y"):
        assert np.array_equal(part[key], full[key][:k])
    assert oracle.orb_detect(pyr, sc["sf"], t=12, edge=19, cap=0)["count"] == full["count"]


# ---------------------------------------------------------------- smoothing
def test_blur_of_an_impulse_is_the_rounded_binomial_product():
    img = np.zeros((30, 30), np.uint8)
    img[15, 14] = 255
    out = oracle.orb_blur(img)
    want = np.zeros((30, 30), np.int64)
    want[12:19, 11:18] = (np.outer(BINOM, BINOM) * 255 + 2048) >> 12
    assert np.array_equal(out, want)


def test_blur_keeps_constants_and_interior_ramps_and_clamps_borders():
    assert np.array_equal(oracle.orb_blur(np.full((20, 25), 93, np.uint8)), np.full((20, 25), 93))
    y, x = np.mgrid[0:40, 0:40]
    ramp = (3 * x + 2 * y + 10).astype(np.uint8)
    out = oracle.orb_blur(ramp).astype(np.int64)
    assert np.array_equal(out[3:-3, 3:-3], ramp[3:-3, 3:-3])
    # column 0, interior rows: the clamped taps repeat column 0
    row = ramp[20].astype(np.int64)
    h = BINOM[:4].sum() * row[0] + BINOM[4] * row[1] + BINOM[5] * row[2] + BINOM[6] * row[3]
    assert out[20, 0] == (h * 64 + 2048) >> 12


# --------------------------------------------------------------- orientation
def ramp_image(kind, n=96):
    y, x = np.mgrid[0:n, 0:n]
    f = {"+x": 2 * x + 20, "+y": 2 * y + 20, "-x": 230 - 2 * x, "-y": 230 - 2 * y,
         "+x+y": x + y + 20, "+x-y": x - y + 120}[kind]
    return f.astype(np.uint8)


@pytest.mark.parametrize("kind,deg", [("+x", 0.0), ("+y", 90.0), ("-x", 180.0), ("-y", 270.0),
                                      ("+x+y", 45.0), ("+x-y", 315.0)])
def test_orientation_of_linear_ramps(kind, deg):
    img = ramp_image(kind)
    pyr = single_level(img)
    kps = {"lx": np.array([48], np.int16), "ly": np.array([48], np.int16), "octave": np.zeros(1, np.uint8)}
    got = oracle.orb_describe(pyr, oracle.orb_blur_pyramid(pyr), kps, synth.orb_pattern())
    assert got["angle"][0] == np.float32(deg)


def test_orientation_disc_has_radius_15_inclusive():
    """m10 of a unit x-ramp is the sum of dx^2 over the disc: an angle of 0
    whatever the disc, so the disc is read off a ramp plus one bright pixel
    placed just inside, then just outside, radius 15."""
    base = ramp_image("+y").astype(np.int32)            # angle 90 exactly
    kps = {"lx": np.array([48], np.int16), "ly": np.array([48], np.int16), "octave": np.zeros(1, np.uint8)}
    pat = synth.orb_pattern()
    for (dx, dy), inside in (((15, 0), True), ((16, 0), False), ((9, 12), True), ((11, 11), False)):
        img = base.copy()
        img[48 + dy, 48 + dx] = 255
        pyr = single_level(img.astype(np.uint8))
        a = oracle.orb_describe(pyr, oracle.orb_blur_pyramid(pyr), kps, pat)["angle"][0]
        assert (a != np.float32(90.0)) == inside, (dx, dy)


def brute_angle(img, u, v):
    yy, xx = np.mgrid[-15:16, -15:16]
    m = xx * xx + yy * yy <= 225
    patch = img[v - 15:v + 16, u - 15:u + 16].astype(np.int64)
    m10, m01 = int((xx * patch)[m].sum()), int((yy * patch)[m].sum())
    return m10, m01


# ---------------------------------------------------------------- descriptor
@pytest.mark.parametrize("kind", ["+x", "+y", "-x", "-y"])
def test_ramp_descriptors_equal_the_pattern_x_order_in_every_direction(kind):
    pat = synth.orb_pattern()
    pyr = single_level(ramp_image(kind))
    kps = {"lx": np.array([48], np.int16), "ly": np.array([48], np.int16), "octave": np.zeros(1, np.uint8)}
    got = oracle.orb_describe(pyr, oracle.orb_blur_pyramid(pyr), kps, pat)
    bits = (pat[:, 0].astype(int) < pat[:, 2].astype(int)).astype(np.uint8)
    assert np.array_equal(got["desc"][0], np.packbits(bits, bitorder="little"))


def test_diagonal_ramp_descriptor_uses_the_exactly_turned_pattern():
    pat = synth.orb_pattern().astype(int)
    pyr = single_level(ramp_image("+x+y"))
    kps = {"lx": np.array([48], np.int16), "ly": np.array([48], np.int16), "octave": np.zeros(1, np.uint8)}
    got = oracle.orb_describe(pyr, oracle.orb_blur_pyramid(pyr), kps, pat.astype(np.int8))
    r = math.sqrt(0.5)

    def turn(x, y):
        c, rr = (x - y) * r, (x + y) * r
        assert abs(abs(c) % 1 - 0.5) > 1e-6 and abs(abs(rr) % 1 - 0.5) > 1e-6
        return math.copysign(math.floor(abs(c) + 0.5), c), math.copysign(math.floor(abs(rr) + 0.5), rr)
    bits = []
    for x1, y1, x2, y2 in pat:
        c1, r1 = turn(x1, y1)
        c2, r2 = turn(x2, y2)
        bits.append(int(c1 + r1 < c2 + r2))             # the image is x + y + 20 there
    assert np.array_equal(got["desc"][0], np.packbits(np.array(bits, np.uint8), bitorder="little"))


def test_descriptors_equal_numpy_brute_force_on_textures():
    """Random keypoints on a textured pyramid: the numpy route (float64
    cos/sin from hypot, round half away from zero) agrees on every test whose
    turned coordinates are not within 1e-9 of a half (those are skipped),
    and the angle agrees with numpy's arctan2 of the numpy moments."""
    sc = synth.scale_tables()
    pyr = oracle.pyramid(texture(9, 240, 320), sc["inv_sf"])
    blurred = oracle.orb_blur_pyramid(pyr)
    rng = np.random.default_rng(10)
    lv = rng.integers(0, 5, 300).astype(np.uint8)
    lx = np.array([rng.integers(19, pyr["width"][l] - 19) for l in lv], np.int16)
    ly = np.array([rng.integers(19, pyr["height"][l] - 19) for l in lv], np.int16)
    pat = synth.orb_pattern()
    got = oracle.orb_describe(pyr, blurred, {"lx": lx, "ly": ly, "octave": lv}, pat)
    checked = 0
    for i in range(300):
        l, w, o = int(lv[i]), int(pyr["width"][lv[i]]), int(pyr["offset"][lv[i]])
        h = int(pyr["height"][l])
        img = pyr["data"][o:o + w * h].reshape(h, w)
        B = blurred[o:o + w * h].reshape(h, w)
        m10, m01 = brute_angle(img, int(lx[i]), int(ly[i]))
        a = math.degrees(math.atan2(m01, m10)) % 360.0
        assert abs(float(got["angle"][i]) - a) < 1e-4 or abs(abs(float(got["angle"][i]) - a) - 360) < 1e-4
        rr = math.hypot(m10, m01)
        c, s = (m10 / rr, m01 / rr) if rr else (1.0, 0.0)
        for t, (x1, y1, x2, y2) in enumerate(pat.astype(int)):
            v = [c * x1 - s * y1, s * x1 + c * y1, c * x2 - s * y2, s * x2 + c * y2]
            if any(abs(abs(q) % 1 - 0.5) < 1e-9 for q in v):
                continue
            q = [int(math.copysign(math.floor(abs(z) + 0.5), z)) for z in v]
            bit = int(B[ly[i] + q[1], lx[i] + q[0]] < B[ly[i] + q[3], lx[i] + q[2]])
            assert (got["desc"][i][t // 8] >> (t % 8)) & 1 == bit, (i, t)
            checked += 1
    assert checked > 0.99 * 300 * 256
