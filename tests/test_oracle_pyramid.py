"""Pins of the oracle's image pyramid (Section IV-B: the pyramid is built on
the device and reused by stereo matching).

Each expected value comes from something other than the oracle: closed forms
that bilinear resampling must reduce to (constant images, linear ramps, exact
2x downscaling), the level sizes of the paper's image shapes, and an
independent vectorised numpy resampler written from the same definition.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth.images import level_sizes

SC = synth.common.scale_tables()


def _level(pyr, l):
    o = int(pyr["offset"][l])
    w, h = int(pyr["width"][l]), int(pyr["height"][l])
    return pyr["data"][o:o + w * h].reshape(h, w)


def _round_half_up_source(x, n_in, n_out):
    """Nearest source pixel of output x (ties up), clamped: exact fractions."""
    s = Fraction(2 * x + 1, 2) * Fraction(n_in, n_out) - Fraction(1, 2)
    s = min(max(s, Fraction(0)), Fraction(n_in - 1))
    return int(np.floor(s + Fraction(1, 2)))


def test_level_sizes_of_the_paper_shapes():
    """752x480 (EuRoC-like) and 512x512 (TUM-VI-like) pyramids hold 1,117,367
    and 811,960 bytes; sizes equal the generator's own rounding of W/sf."""
    for (W, H), total in (((752, 480), 1117367), ((512, 512), 811960)):
        lay = oracle.pyramid_layout(W, H, SC["inv_sf"])
        assert lay["bytes"] == total
        ws, hs = level_sizes(W, H, SC)
        assert list(lay["width"]) == ws and list(lay["height"]) == hs
        assert lay["offset"][0] == 0
        assert all(lay["offset"][l + 1] - lay["offset"][l] == ws[l] * hs[l] for l in range(7))
    lay = oracle.pyramid_layout(752, 480, SC["inv_sf"])
    assert (lay["width"][7], lay["height"][7]) == (210, 134)


@pytest.mark.parametrize("c", [0, 1, 77, 254, 255])
def test_constant_image_gives_constant_levels(c):
    img = np.full((61, 83), c, np.uint8)
    pyr = oracle.pyramid(img, SC["inv_sf"])
    assert (pyr["data"] == c).all()
    assert (_level(pyr, 0) == img).all()


@pytest.mark.parametrize("W,H", [(200, 37), (96, 64), (255, 9)])
def test_horizontal_ramp_is_round_half_up_of_the_source_column(W, H):
    """I(x, y) = x: bilinear weights on a unit ramp give x0 + [frac >= 1/2],
    i.e. the exact source coordinate rounded half up."""
    img = np.tile(np.arange(W, dtype=np.uint8), (H, 1))
    pyr = oracle.pyramid(img, SC["inv_sf"])
    for l in range(1, 8):
        lv = _level(pyr, l)
        want = np.array([_round_half_up_source(x, W, lv.shape[1]) for x in range(lv.shape[1])])
        assert (lv == want[None, :]).all(), l


@pytest.mark.parametrize("W,H", [(40, 250), (7, 96)])
def test_vertical_ramp_is_round_half_up_of_the_source_row(W, H):
    img = np.tile(np.arange(H, dtype=np.uint8)[:, None], (1, W))
    pyr = oracle.pyramid(img, SC["inv_sf"])
    for l in range(1, 8):
        lv = _level(pyr, l)
        want = np.array([_round_half_up_source(y, H, lv.shape[0]) for y in range(lv.shape[0])])
        assert (lv == want[:, None]).all(), l


def test_exact_halving_is_the_rounded_box_average():
    """With inv_sf = 1/2 the source centre of every output pixel sits midway
    between four pixels: the level is (p00 + p01 + p10 + p11 + 2) >> 2."""
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (48, 64), dtype=np.uint8)
    inv = np.array([1.0, 0.5], np.float32)
    pyr = oracle.pyramid(img, inv)
    lv = _level(pyr, 1)
    s = img.astype(np.int64)
    box = s[0::2, 0::2] + s[0::2, 1::2] + s[1::2, 0::2] + s[1::2, 1::2]
    assert lv.shape == (24, 32)
    assert (lv == (box + 2) >> 2).all()


def _numpy_level(img, w, h):
    """Bilinear resample written independently with numpy (vectorised over
    the whole level), from the definition in the oracle's header."""
    H, W = img.shape

    def taps(n_in, n_out):
        x = np.arange(n_out, dtype=np.int64)
        num = (2 * x + 1) * n_in - n_out
        den = 2 * n_out
        i0 = np.where(num > 0, num // den, 0)
        wt = np.where(num > 0, (256 * (num % den)) // den, 0)
        past = i0 >= n_in - 1
        i0 = np.where(past, n_in - 1, i0)
        wt = np.where(past, 0, wt)
        return i0, np.minimum(i0 + 1, n_in - 1), wt

    x0, x1, a = taps(W, w)
    y0, y1, b = taps(H, h)
    I = img.astype(np.int64)
    top = (256 - a)[None, :] * I[y0][:, x0] + a[None, :] * I[y0][:, x1]
    bot = (256 - a)[None, :] * I[y1][:, x0] + a[None, :] * I[y1][:, x1]
    v = (256 - b)[:, None] * top + b[:, None] * bot
    return ((v + 32768) >> 16).astype(np.uint8)


@pytest.mark.parametrize("W,H,seed", [(752, 480, 4), (512, 512, 5), (101, 67, 6), (17, 300, 7)])
def test_random_images_match_numpy_resampler(W, H, seed):
    img = np.random.default_rng(seed).integers(0, 256, (H, W), dtype=np.uint8)
    pyr = oracle.pyramid(img, SC["inv_sf"])
    assert (_level(pyr, 0) == img).all()
    for l in range(1, 8):
        lv = _level(pyr, l)
        assert (lv == _numpy_level(img, lv.shape[1], lv.shape[0])).all(), l


def test_levels_stay_between_the_neighbouring_pixels():
    """Every output value lies between the min and max of its 2x2 source taps
    (a convex combination, rounded)."""
    img = np.random.default_rng(8).integers(0, 256, (120, 160), dtype=np.uint8)
    pyr = oracle.pyramid(img, SC["inv_sf"])
    for l in range(1, 8):
        lv = _level(pyr, l).astype(int)
        h, w = lv.shape
        for y in range(0, h, 7):
            ys = _round_half_up_source(y, 120, h)
            for x in range(0, w, 5):
                xs = _round_half_up_source(x, 160, w)
                blk = img[max(ys - 1, 0):ys + 2, max(xs - 1, 0):xs + 2].astype(int)
                assert blk.min() <= lv[y, x] <= blk.max()
