"""The seeded workloads (plus tiny variants for brute-force checks).

Each workload has its own master seed, 10757000 + a fixed offset; sub-seeds come
from SeedSequence.spawn.
  pinhole_frame_1200      one pinhole stereo frame, 752x480, 1200 kp/image,
                          3000 map points, 64x48 grid (offset 1)
  fisheye_frame_1500      one fisheye stereo frame, 512x512, 1500 kp/image,
                          5000 map points (offset 2)
  clustered_search_20000  local-map search only: 20000 clustered map points,
                          3000 kp, 96x64 grid (offset 3)
  mixed_batch             64 frames, 32 pinhole + 32 fisheye in seeded order,
                          kp ~ U{300..3000}, map ~ U{1000..20000} (offset 4)
  clustered_batch         the clustered scene over 64 seeds spawned from offset 3
"""
from __future__ import annotations

import numpy as np

from .clustered import clustered_frame
from .common import MASTER_SEED
from .fisheye import fisheye_frame
from .pinhole import pinhole_camera, pinhole_frame


def seed_of(offset: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(MASTER_SEED + offset)


def pinhole_frame_1200(seed=None):
    return [pinhole_frame(seed if seed is not None else seed_of(1))]


def fisheye_frame_1500(seed=None):
    return [fisheye_frame(seed if seed is not None else seed_of(2))]


def clustered_search_20000(seed=None):
    return [clustered_frame(seed if seed is not None else seed_of(3))]


def mixed_batch(seed=None, n_frames: int = 64):
    ss = seed if seed is not None else seed_of(4)
    ctl_ss, *frame_ss = ss.spawn(n_frames + 1)
    rng = np.random.default_rng(ctl_ss)
    kinds = np.array(["pinhole"] * (n_frames // 2) + ["fisheye"] * (n_frames - n_frames // 2))
    rng.shuffle(kinds)
    n_kp = rng.integers(300, 3001, n_frames)
    n_map = rng.integers(1000, 20001, n_frames)
    frames = []
    for i in range(n_frames):
        if kinds[i] == "pinhole":
            frames.append(pinhole_frame(frame_ss[i], n_kp=int(n_kp[i]), n_map=int(n_map[i])))
        else:
            frames.append(fisheye_frame(frame_ss[i], n_kp=int(n_kp[i]), n_map=int(n_map[i])))
    return frames


def clustered_batch(seed=None, n_frames: int = 64):
    """The clustered local-map scene (20000 map points, 3000 keypoints, 96x64
    grid) over `n_frames` seeds, for one batched submission."""
    ss = seed if seed is not None else seed_of(3)
    return [clustered_frame(s) for s in ss.spawn(n_frames)]


def tiny_pinhole(seed, n_kp: int = 80, n_map: int = 120, grid=(12, 8)):
    cam = pinhole_camera(W=240, H=160, fx=140.0, cx=120.0, cy=80.0, b=0.11)
    return pinhole_frame(seed, n_kp=n_kp, n_map=n_map, grid=grid, cam=cam)


def tiny_fisheye(seed, n_kp: int = 80, n_map: int = 120, grid=(12, 8)):
    return fisheye_frame(seed, n_kp=n_kp, n_map=n_map, grid=grid)


def tiny_clustered(seed, n_map: int = 400, n_kp: int = 120, grid=(16, 12)):
    return clustered_frame(seed, n_map=n_map, n_kp=n_kp, n_blobs=4, grid=grid)


SINGLE_FRAME = {"pinhole_frame_1200": pinhole_frame_1200, "fisheye_frame_1500": fisheye_frame_1500,
                "clustered_search_20000": clustered_search_20000}


def workload(name: str):
    return SINGLE_FRAME[name]()
