"""Device image pyramid (ft_build_pyramid, and batch jobs that build their
pyramids before stereo) against the CPU oracle, byte for byte.

Sizes: the two image shapes of the workloads (752x480, 512x512), odd widths,
rows padded past the width, a source not 4-byte aligned, the smallest image
every level of which is non-empty, and the widest image the build accepts.
A batch of pinhole frames whose pyramids are built on the device gives the
oracle's stereo and search results on the oracle's pyramids of the same
level-0 images.
"""
import copy
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity import compare_frame

pytestmark = pytest.mark.gpu

SC = synth.scale_tables()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(ft):
    return ft.Context(ft.default_limits(max_batch_frames=16, max_map_points=32768))


def _device_build(ft, ctx, img, pitch=None, shift=0):
    """Build the pyramid of host image `img` on the device; the source rows
    sit `pitch` bytes apart, `shift` bytes past an aligned allocation."""
    H, W = img.shape
    pitch = pitch or W
    buf = np.full(shift + pitch * H, 0x5A, np.uint8)
    for y in range(H):
        buf[shift + y * pitch: shift + y * pitch + W] = img[y]
    src = torch.from_numpy(buf).cuda()
    scales = ft._scales(SC)
    lay, nbytes = ft.pyramid_layout(W, H, scales)
    out = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    lay.data = out.data_ptr()
    image = ft.ft_image(src.data_ptr() + shift, W, H, pitch)
    ctx.ft_build_pyramid(image, scales, lay)
    torch.cuda.synchronize()
    return out.cpu().numpy(), lay


@pytest.mark.parametrize("W,H,pitch,shift,seed", [
    (752, 480, None, 0, 1), (512, 512, None, 0, 2), (101, 67, None, 0, 3), (17, 300, None, 0, 4),
    (640, 480, 704, 0, 5), (255, 129, 260, 3, 6), (2, 2, None, 0, 7), (3, 97, 5, 1, 8), (1536, 96, None, 0, 9)])
def test_pyramid_equals_oracle(ft, ctx, W, H, pitch, shift, seed):
    say("pyramid", W, H, "pitch", pitch, "shift", shift)
    img = np.random.default_rng(seed).integers(0, 256, (H, W), dtype=np.uint8)
    got, lay = _device_build(ft, ctx, img, pitch, shift)
    want = oracle.pyramid(img, SC["inv_sf"])
    assert list(lay.offset) == list(want["offset"]) and list(lay.width) == list(want["width"])
    assert got.size == want["data"].size
    bad = np.nonzero(got != want["data"])[0]
    assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:8].tolist()}"


def test_pyramid_of_a_workload_image(ft, ctx):
    """Level 0 of a generated pinhole frame (band-limited texture)."""
    f = synth.tiny_pinhole(11)
    pyr = f["pyr_left"]
    w, h = int(pyr["width"][0]), int(pyr["height"][0])
    img = pyr["data"][:w * h].reshape(h, w)
    got, _ = _device_build(ft, ctx, img)
    assert np.array_equal(got, oracle.pyramid(img, SC["inv_sf"])["data"])


def test_pyramid_rejects_bad_inputs(ft, ctx):
    scales = ft._scales(SC)
    src = torch.zeros(2000 * 8, dtype=torch.uint8, device="cuda")
    lay, nbytes = ft.pyramid_layout(64, 48, scales)
    out = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    lay.data = out.data_ptr()
    bad = ft.ft_image(src.data_ptr(), 64, 48, 32)                 # pitch below the width
    assert ctx.ft_build_pyramid(bad, scales, lay, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    wide = ft.ft_image(src.data_ptr(), 2000, 8, 2000)              # wider than the staged rows allow
    lay2, n2 = ft.pyramid_layout(2000, 8, scales)
    lay2.data = out.data_ptr()
    assert ctx.ft_build_pyramid(wide, scales, lay2, check=False) == ft.FT_ERR_CAPACITY
    ok = ft.ft_image(src.data_ptr(), 64, 48, 64)
    lay.width[3] += 1                                              # not the packed layout
    assert ctx.ft_build_pyramid(ok, scales, lay, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    with pytest.raises(ft.FtError):
        ft.pyramid_layout(1, 1, scales)                            # level 7 would be empty
    torch.cuda.synchronize()


@pytest.mark.parametrize("n_frames", [1, 6])
def test_batch_builds_pyramids_before_stereo(ft, ctx, n_frames):
    """Pinhole jobs with build_pyramids: the device pyramids equal the
    oracle's, and stereo + search equal the oracle on the oracle's pyramids;
    fisheye jobs in the same batch are unaffected."""
    frames = synth.mixed_batch(n_frames=2 * n_frames)[:2 * n_frames]
    ref_frames, dfs = [], []
    for f in frames:
        g = copy.copy(f)
        if f["kind"] == "pinhole":
            for side in ("left", "right"):
                pyr = f["pyr_" + side]
                w, h = int(pyr["width"][0]), int(pyr["height"][0])
                g["pyr_" + side] = oracle.pyramid(pyr["data"][:w * h].reshape(h, w), SC["inv_sf"])
        ref_frames.append(g)
        dfs.append(ft.DeviceFrame(f, "cuda", build_pyramids=True))
    say("batch of", len(frames), "frames,", sum(d.build_pyramids for d in dfs), "building pyramids")
    for mode in (ft.FT_EXEC_EAGER, ft.FT_EXEC_GRAPH):
        ctx.ft_set_exec_mode(mode)
        ctx.ft_batch_wait(ctx.ft_batch_submit([d.job() for d in dfs]))
        torch.cuda.synchronize()
        for g, d in zip(ref_frames, dfs):
            if d.build_pyramids:
                pyrs = d.pyramids()
                for side in ("left", "right"):
                    assert np.array_equal(pyrs[side], g["pyr_" + side]["data"]), side
            compare_frame(d.results(), oracle.run_frame(g))
    ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
