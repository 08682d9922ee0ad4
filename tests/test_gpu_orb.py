"""ORB extraction on the device against the CPU oracle (Section II-A,
Section IV-B): corners (count, order, level coordinates, scores, level-0
coordinates) and the smoothed pyramid byte for byte; descriptors bit for bit
and orientations within 1e-4 degrees; on full-size EuRoC-like pyramids,
ragged small images, capacity limits, host-filtered subsets, keypoints too
close to a border, a device-built pyramid, and invalid arguments."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.test_oracle_orb import texture

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(ft):
    return ft.Context(ft.default_limits(max_batch_frames=1, max_inflight=1))


@pytest.fixture(scope="module")
def scales(ft):
    return ft._scales(synth.scale_tables())


def _angles_close(got, want):
    d = np.abs(got.astype(np.float64) - want.astype(np.float64))
    d = np.minimum(d, 360.0 - d)
    assert d.max(initial=0.0) < 1e-4, float(d.max(initial=0.0))


def _check(ft, ctx, scales, pyr, t, pattern, capacity=None, tag=""):
    sc = synth.scale_tables()
    want = oracle.orb_detect(pyr, sc["sf"], t=t, edge=19)
    cap = capacity if capacity is not None else max(want["count"], 1)
    d = ft.DeviceOrb(pyr, capacity=cap)
    say("orb", tag, "t", t, "corners", want["count"], "capacity", cap)
    d.detect(ctx, scales, threshold=t, edge=19)
    d.describe(ctx, pattern)
    torch.cuda.synchronize()
    got = d.results()
    assert got["count"] == want["count"], tag
    k = min(cap, want["count"])
    for key in ("lx", "ly", "octave", "score", "x", "y"):
        assert np.array_equal(got[key], want[key][:k]), (tag, key)
    blurred = oracle.orb_blur_pyramid(pyr)
    assert np.array_equal(d.blurred.cpu().numpy(), blurred), tag
    wd = oracle.orb_describe(pyr, blurred, {key: want[key][:k] for key in ("lx", "ly", "octave")}, pattern)
    assert np.array_equal(got["desc"], wd["desc"]), tag
    _angles_close(got["angle"], wd["angle"])
    return got


@pytest.mark.parametrize("t", [20, 12])
def test_full_size_pinhole_pyramids_equal_oracle(ft, ctx, scales, t):
    f = synth.pinhole_frame_1200()[0]
    pat = synth.orb_pattern()
    for side in ("pyr_left", "pyr_right"):
        got = _check(ft, ctx, scales, f[side], t, pat, tag=side)
        assert got["count"] > 1000


@pytest.mark.parametrize("h,w,seed", [(61, 97, 1), (77, 130, 2), (240, 333, 3)])
def test_ragged_small_images_equal_oracle(ft, ctx, scales, h, w, seed):
    sc = synth.scale_tables()
    pyr = oracle.pyramid(texture(seed, h, w), sc["inv_sf"])
    _check(ft, ctx, scales, pyr, 15, synth.orb_pattern(), tag=f"{h}x{w}")


def test_capacity_keeps_the_first_corners(ft, ctx, scales):
    f = synth.pinhole_frame_1200()[0]
    sc = synth.scale_tables()
    n = oracle.orb_detect(f["pyr_left"], sc["sf"], t=20, edge=19)["count"]
    _check(ft, ctx, scales, f["pyr_left"], 20, synth.orb_pattern(), capacity=n // 3, tag="third")
    d = ft.DeviceOrb(f["pyr_left"], capacity=0)
    d.detect(ctx, scales, threshold=20, edge=19)
    torch.cuda.synchronize()
    assert int(d.t["count"][0]) == n


def test_hand_built_images_equal_oracle(ft, ctx, scales):
    sc = synth.scale_tables()
    img = np.full((120, 160), 60, np.uint8)
    img[40, 50] = 220
    img[80:, 100:] = 200                      # a bright quadrant: corners at its corner only
    img[70, 30] = img[70, 31] = 180           # a plateau of two equal corners
    _check(ft, ctx, scales, oracle.pyramid(img, sc["inv_sf"]), 20, synth.orb_pattern(), tag="hand")


def test_device_built_pyramid_then_orb(ft, ctx, scales):
    """Level 0 uploaded, pyramid built on the device, then detection and
    description on it: equal to the oracle's pyramid and extraction."""
    f = synth.pinhole_frame_1200()[0]
    pl = f["pyr_left"]
    W, H = int(pl["width"][0]), int(pl["height"][0])
    img0 = pl["data"][:W * H].reshape(H, W)
    sc = synth.scale_tables()
    want_pyr = oracle.pyramid(img0, sc["inv_sf"])
    lay, nbytes = ft.pyramid_layout(W, H, scales)
    dev_img = torch.from_numpy(np.ascontiguousarray(img0)).cuda()
    dev_pyr = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    lay.data = dev_pyr.data_ptr()
    ctx.ft_build_pyramid(ft.ft_image(dev_img.data_ptr(), W, H, W), scales, lay)
    pyr = {"data": dev_pyr, "offset": np.array(lay.offset), "width": np.array(lay.width),
           "height": np.array(lay.height)}
    d = ft.DeviceOrb(pyr, capacity=65536)
    pat = synth.orb_pattern()
    d.detect(ctx, scales)
    d.describe(ctx, pat)
    torch.cuda.synchronize()
    assert np.array_equal(dev_pyr.cpu().numpy(), want_pyr["data"])
    want = oracle.orb_detect(want_pyr, sc["sf"], t=20, edge=19)
    got = d.results()
    assert got["count"] == want["count"]
    for key in ("lx", "ly", "octave", "score"):
        assert np.array_equal(got[key], want[key]), key
    wd = oracle.orb_describe(want_pyr, oracle.orb_blur_pyramid(want_pyr), want, pat)
    assert np.array_equal(got["desc"], wd["desc"])


def test_describe_of_a_host_filtered_subset_and_border_keypoints(ft, ctx, scales):
    """Every third corner (the caller's filtering), plus keypoints too close
    to their level's border or of a level beyond the pyramid: the valid ones
    equal the oracle, the others get angle -1 and a zero descriptor."""
    f = synth.pinhole_frame_1200()[0]
    pyr = f["pyr_left"]
    sc = synth.scale_tables()
    pat = synth.orb_pattern()
    allc = oracle.orb_detect(pyr, sc["sf"], t=20, edge=19)
    sub = {k: allc[k][::3] for k in ("lx", "ly", "octave")}
    bad_lx = np.array([14, 20, 30, int(pyr["width"][2]) - 15], np.int16)
    bad_ly = np.array([40, 14, 30, 40], np.int16)
    bad_oct = np.array([0, 1, 9, 2], np.uint8)
    lx = np.concatenate([sub["lx"], bad_lx]); ly = np.concatenate([sub["ly"], bad_ly])
    oc = np.concatenate([sub["octave"], bad_oct])
    n = len(lx)
    d = ft.DeviceOrb(pyr, capacity=8)
    d.detect(ctx, scales)                    # fills the smoothed pyramid
    dev = {"lx": torch.from_numpy(lx).cuda(), "ly": torch.from_numpy(ly).cuda(), "oct": torch.from_numpy(oc).cuda()}
    angle = torch.empty(n, dtype=torch.float32, device="cuda")
    desc = torch.full((n, 32), 0xAB, dtype=torch.uint8, device="cuda")
    ctx.ft_orb_describe(d.pyr, d.blurred.data_ptr(), n, None, dev["lx"].data_ptr(), dev["ly"].data_ptr(),
                        dev["oct"].data_ptr(), pat, angle.data_ptr(), desc.data_ptr())
    torch.cuda.synchronize()
    m = len(sub["lx"])
    wd = oracle.orb_describe(pyr, oracle.orb_blur_pyramid(pyr), sub, pat)
    assert np.array_equal(desc[:m].cpu().numpy(), wd["desc"])
    _angles_close(angle[:m].cpu().numpy(), wd["angle"])
    assert np.all(angle[m:].cpu().numpy() == -1.0)
    assert not desc[m:].cpu().numpy().any()


def test_invalid_arguments_are_rejected(ft, ctx, scales):
    f = synth.pinhole_frame_1200()[0]
    d = ft.DeviceOrb(f["pyr_left"], capacity=16)
    for t, e in ((0, 19), (255, 19), (20, 18)):
        assert d.detect(ctx, scales, threshold=t, edge=e, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    bad = synth.orb_pattern().copy()
    bad[7] = (10, 10, 0, 0)                   # 10^2 + 10^2 > 13^2
    assert d.describe(ctx, bad, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    wide = ft.ft_pyramid.from_buffer_copy(bytes(d.pyr))
    wide.width[0] = ft.FT_PYRAMID_MAX_WIDTH + 1
    c = d.corners
    assert ctx.ft_orb_detect(wide, scales, ft.ft_orb_params(20, 19), d.blurred.data_ptr(), c,
                             check=False) == ft.FT_ERR_CAPACITY
    mis = ft.ft_orb_corners.from_buffer_copy(bytes(c))
    mis.x = c.x + 2
    assert ctx.ft_orb_detect(d.pyr, scales, ft.ft_orb_params(20, 19), None, mis,
                             check=False) == ft.FT_ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
