"""Seeded inputs of the last-frame search by projection (Initial Pose
Estimation: the previous frame's matched map points are projected into the
current frame and matched against its keypoints).

A case is built on a current frame from the other generators: the last-frame
points are the map points behind the frame's true keypoints plus map points
without one (20% more); the last-frame octave of a true point is its current
keypoint's octave, moved by one level with probability 0.3; orientations of
last-frame keypoints are uniform, and a true current keypoint's orientation is
the last one turned by the frame-to-frame image rotation plus noise, while
every other keypoint's orientation is uniform, as is that of 10% of the true
keypoints (matches the rotation check should drop).  Pinhole cases carry a stereo
right coordinate for true keypoints (truth disparity plus noise, -1 elsewhere).
"""
from __future__ import annotations

import numpy as np

from . import common as C


def motion_params(th: float = 7.0, direction: int = 0, check_orientation: int = 1, bins: int = 30):
    """Constants of the last-frame search (values restated from the ORB-SLAM3
    tracking the paper accelerates: stereo search radius 7 * scale, distance
    threshold 100, 30 rotation bins)."""
    return {"th": th, "th_high": 100, "direction": direction,
            "check_orientation": check_orientation, "bins": bins}


def last_frame_case(frame: dict, seed, rot_deg: float = 5.0, angle_sd: float = 3.0,
                    extra_frac: float = 0.2, wrong_angle_frac: float = 0.1, direction: int = 0,
                    th: float = 7.0, view: int = 0, check_orientation: int = 1) -> dict:
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    r_pick, r_oct, r_ang, r_ur = [np.random.default_rng(s) for s in ss.spawn(4)]
    spec = frame["search"][view]
    kp = frame[spec["image"]]
    nK = len(kp["x"])
    mp = frame["map"]
    nM = len(mp["dmin"])
    pairs = frame["truth"]["map_kp"]
    if spec["image"] != "left":
        pairs = pairs[:0]
    m_true, k_true = pairs[:, 0], pairs[:, 1]
    others = np.setdiff1d(np.arange(nM), m_true)
    n_extra = min(len(others), int(round(extra_frac * len(m_true))))
    m_extra = r_pick.choice(others, n_extra, replace=False)
    m_all = np.concatenate([m_true, m_extra])
    order = r_pick.permutation(len(m_all))
    m_all = m_all[order]
    is_true = np.concatenate([np.ones(len(m_true), bool), np.zeros(n_extra, bool)])[order]
    k_of = np.concatenate([k_true, np.full(n_extra, -1)])[order]

    n_last = len(m_all)
    step = np.where(r_oct.random(n_last) < 0.5, -1, 1)
    move = r_oct.random(n_last) < 0.3
    cur_oct = np.where(is_true, kp["octave"][np.maximum(k_of, 0)].astype(np.int64), 0)
    lo = np.where(is_true, np.clip(cur_oct + np.where(move, step, 0), 0, C.N_LEVELS - 1),
                  r_oct.integers(0, C.N_LEVELS, n_last))
    la = r_ang.uniform(0.0, 360.0, n_last).astype(np.float32)
    ka = r_ang.uniform(0.0, 360.0, nK).astype(np.float32)
    turned = np.mod(la[is_true].astype(np.float64) - rot_deg + r_ang.normal(0.0, angle_sd, is_true.sum()), 360.0)
    wrong = r_ang.random(is_true.sum()) < wrong_angle_frac   # a keypoint whose orientation is off
    turned = np.where(wrong, r_ang.uniform(0.0, 360.0, is_true.sum()), turned)
    ka[k_of[is_true]] = turned.astype(np.float32)

    u_right = None
    if frame["kind"] == "pinhole" and spec.get("use_u_right"):
        d = frame["truth"]["disparity"]
        left_idx = frame["truth"]["stereo_pairs"][:, 0]
        u_right = np.full(nK, -1.0, np.float32)
        u_right[left_idx] = (kp["x"][left_idx].astype(np.float64) - d +
                             r_ur.uniform(-0.3, 0.3, len(left_idx))).astype(np.float32)

    return {
        "kind": "last_frame",
        "scales": frame["scales"],
        "last": {"pos": np.ascontiguousarray(mp["pos"][m_all]),
                 "desc": np.ascontiguousarray(mp["desc"][m_all]),
                 "octave": lo.astype(np.uint8), "angle": la},
        "kps": {**{k: kp[k] for k in ("x", "y", "octave", "desc")}, "angle": ka},
        "cam": spec["cam"],
        "grid": spec["grid"],
        "preassigned": spec.get("preassigned"),
        "u_right": u_right,
        "params": motion_params(th, direction, check_orientation),
        "truth": {"last_kp": np.stack([np.nonzero(is_true)[0], k_of[is_true]], axis=1)},
    }
