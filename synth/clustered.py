"""Seeded local-map tracking scene at scale: a clustered map and one frame.

20000 map points in 40 Gaussian blobs (sigma 0.5 m) whose centres are uniform
in a 1-15 m pinhole frustum; 3000 keypoints, of which 2400 are projections of
map points under the true pose (level = predicted level +- 1) and 600 are
distractors.  The search pose is the true pose perturbed by 2 cm / 0.5 deg.
"""
from __future__ import annotations

import numpy as np

from . import common as C
from .pinhole import back_project, pinhole_camera


def _in_frustum(P, cam, zlo=1.0, zhi=15.0):
    z = P[:, 2]
    zs = np.where(z > 0, z, 1.0)
    u = float(cam["fx"]) * P[:, 0] / zs + float(cam["cx"])
    v = float(cam["fy"]) * P[:, 1] / zs + float(cam["cy"])
    return (z >= zlo) & (z <= zhi) & (u >= 0) & (u < cam["W"]) & (v >= 0) & (v < cam["H"])


def clustered_frame(seed, n_map: int = 20000, n_kp: int = 3000, n_blobs: int = 40,
                    sigma: float = 0.5, grid=(96, 64), th: float = 2.0):
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    r_map, r_kp, r_desc, r_pose = [np.random.default_rng(s) for s in ss.spawn(4)]
    cam = pinhole_camera()
    W, H = cam["W"], cam["H"]
    sc = C.scale_tables()
    sf = sc["sf"].astype(np.float64)

    centres = back_project(r_map.uniform(0, W, n_blobs), r_map.uniform(0, H, n_blobs),
                           r_map.uniform(1.0, 15.0, n_blobs), cam)
    blob = r_map.integers(0, n_blobs, n_map)
    P = centres[blob] + r_map.normal(0, sigma, (n_map, 3))
    for _ in range(1000):
        bad = ~_in_frustum(P, cam)
        if not bad.any():
            break
        P[bad] = centres[blob[bad]] + r_map.normal(0, sigma, (int(bad.sum()), 3))
    o_ref = r_map.integers(0, C.N_LEVELS, n_map)
    mdesc = C.random_descriptors(r_desc, n_map)
    mp = C.map_point_fields(r_map, P, np.zeros(3), o_ref, sc, mdesc)

    n_true = int(round(0.8 * n_kp))
    src = r_kp.choice(n_map, n_true, replace=False)
    lv = np.clip(o_ref[src] + r_kp.integers(-1, 2, n_true), 0, C.N_LEVELS - 1)
    Ps = P[src]
    u = float(cam["fx"]) * Ps[:, 0] / Ps[:, 2] + float(cam["cx"])
    v = float(cam["fy"]) * Ps[:, 1] / Ps[:, 2] + float(cam["cy"])
    x = np.clip(np.rint(u / sf[lv]) * sf[lv], 0, W - 1)
    y = np.clip(np.rint(v / sf[lv]) * sf[lv], 0, H - 1)
    n_dis = n_kp - n_true
    lv_d = r_kp.integers(0, C.N_LEVELS, n_dis)
    xd = np.rint(r_kp.uniform(0, W - 1, n_dis) / sf[lv_d]) * sf[lv_d]
    yd = np.rint(r_kp.uniform(0, H - 1, n_dis) / sf[lv_d]) * sf[lv_d]
    kp = {"x": np.concatenate([x, np.clip(xd, 0, W - 1)]).astype(np.float32),
          "y": np.concatenate([y, np.clip(yd, 0, H - 1)]).astype(np.float32),
          "octave": np.concatenate([lv, lv_d]).astype(np.uint8),
          "desc": np.concatenate([C.flip_bits(r_desc, mdesc[src], r_desc.integers(0, 25, n_true)),
                                  C.random_descriptors(r_desc, n_dis)])}
    perm = r_kp.permutation(n_kp)
    kp = C.permute_keypoints(kp, perm)
    inv = np.argsort(perm)

    R_cw, t_cw, O_w = C.perturbed_pose(r_pose, np.eye(3), np.zeros(3))
    return {
        "kind": "search",
        "scales": sc,
        "left": kp,
        "map": mp,
        "search": [{
            "cam": {"model": 0, "fx": cam["fx"], "fy": cam["fy"], "cx": cam["cx"],
                    "cy": cam["cy"], "k": np.zeros(4, np.float32), "bf": cam["bf"],
                    "bounds": np.array([0, W, 0, H], np.float32),
                    **C.pose_dict(R_cw, t_cw, O_w)},
            "image": "left", "grid": tuple(grid),
            "preassigned": np.zeros(n_kp, np.uint8), "use_u_right": False}],
        "search_params": C.search_params(th),
        "truth": {"map_kp": np.stack([src, inv[:n_true]], axis=1)},
        "size": {"W": W, "H": H},
    }
