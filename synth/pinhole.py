"""Seeded rectified-pinhole stereo frame with its local map.

Shaped like an EuRoC stereo-inertial frame (752x480, fx = 435, b = 0.11 m):
keypoints are placed on pyramid levels with the ORB per-level budget, 80% of
them as true left/right pairs along the disparity field and 20% as distractors
with random positions and descriptors.  The local map holds points
back-projected from true left keypoints plus points uniform in a 1-15 m
frustum.  Everything is generated in float64 and stored as float32.
"""
from __future__ import annotations

import numpy as np

from . import common as C
from .images import DisparityField, level_sizes, noise_texture, pyramid, right_image

BORDER = 16


def pinhole_camera(W=752, H=480, fx=435.0, cx=367.0, cy=248.0, b=0.11):
    fx32 = np.float32(fx)
    b32 = np.float32(b)
    return {"W": W, "H": H, "fx": fx32, "fy": fx32, "cx": np.float32(cx),
            "cy": np.float32(cy), "b": b32, "bf": np.float32(fx32 * b32)}


def _sample_level_pixels(rng, level, ws, hs, border=BORDER):
    xl = np.array([rng.integers(border, ws[l] - border) for l in level], np.int64)
    yl = np.array([rng.integers(border, hs[l] - border) for l in level], np.int64)
    return xl, yl


def _levels_from_alloc(rng, n):
    alloc = C.level_allocation(n)
    lv = np.repeat(np.arange(C.N_LEVELS), alloc)
    rng.shuffle(lv)
    return lv


def back_project(u, v, Z, cam):
    return np.stack([(u - float(cam["cx"])) * Z / float(cam["fx"]),
                     (v - float(cam["cy"])) * Z / float(cam["fy"]), Z], axis=1)


def pinhole_frame(seed, n_kp: int = 1200, n_map: int = 3000, grid=(64, 48),
                  cam: dict | None = None, th: float = 2.0,
                  preassigned_frac: float = 0.1, images: bool = True):
    """One pinhole stereo frame: images, pyramids, keypoints, local map.

    `seed` is an int or a numpy SeedSequence.
    """
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    r_img, r_kp, r_desc, r_map, r_pose = [np.random.default_rng(s) for s in ss.spawn(5)]
    cam = cam or pinhole_camera()
    W, H = cam["W"], cam["H"]
    sc = C.scale_tables()
    ws, hs = level_sizes(W, H, sc)
    sf = sc["sf"].astype(np.float64)

    left_img = noise_texture(r_img, H, W)
    field = DisparityField(r_img, W, H)
    right_img = right_image(r_img, left_img, field)

    # ---- keypoints -------------------------------------------------------
    levels = _levels_from_alloc(r_kp, n_kp)
    n_true = int(round(0.8 * n_kp))
    lv_true = levels[:n_true]
    lv_dis_l = levels[n_true:]

    xL = np.zeros(n_true, np.float32)
    yL = np.zeros(n_true, np.float32)
    xR = np.zeros(n_true, np.float32)
    yR = np.zeros(n_true, np.float32)
    lvR = np.zeros(n_true, np.int64)
    d_true = np.zeros(n_true)
    todo = np.arange(n_true)
    for _ in range(200):
        if todo.size == 0:
            break
        l = lv_true[todo]
        xl, yl = _sample_level_pixels(r_kp, l, ws, hs)
        x0 = (xl * sf[l]).astype(np.float32)
        y0 = (yl * sf[l]).astype(np.float32)
        xr_real = field.right_x(x0.astype(np.float64), y0.astype(np.float64))
        same = r_kp.random(todo.size) < 0.85
        step = np.where(r_kp.random(todo.size) < 0.5, -1, 1)
        lr = np.where(same, l, np.clip(l + step, 0, C.N_LEVELS - 1))
        xr_l = np.rint(xr_real / sf[lr]).astype(np.int64)
        yr_l = np.rint(y0 / sf[lr]).astype(np.int64) + r_kp.integers(-1, 2, todo.size)
        wl = np.array([ws[k] for k in lr])
        hl = np.array([hs[k] for k in lr])
        ok = ((xr_l >= BORDER) & (xr_l < wl - BORDER) &
              (yr_l >= BORDER) & (yr_l < hl - BORDER))
        idx = todo[ok]
        xL[idx], yL[idx] = x0[ok], y0[ok]
        xR[idx] = (xr_l[ok] * sf[lr[ok]]).astype(np.float32)
        yR[idx] = (yr_l[ok] * sf[lr[ok]]).astype(np.float32)
        lvR[idx] = lr[ok]
        d_true[idx] = x0[ok].astype(np.float64) - xr_real[ok]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("could not place true stereo pairs")

    base = C.random_descriptors(r_desc, n_true)
    dL_true = base
    dR_true = C.flip_bits(r_desc, base, r_desc.integers(0, 25, n_true))

    n_dis = n_kp - n_true
    lv_dis_r = _levels_from_alloc(r_kp, n_kp)[:n_dis]
    xdl, ydl = _sample_level_pixels(r_kp, lv_dis_l, ws, hs)
    xdr, ydr = _sample_level_pixels(r_kp, lv_dis_r, ws, hs)

    left = {"x": np.concatenate([xL, (xdl * sf[lv_dis_l]).astype(np.float32)]),
            "y": np.concatenate([yL, (ydl * sf[lv_dis_l]).astype(np.float32)]),
            "octave": np.concatenate([lv_true, lv_dis_l]).astype(np.uint8),
            "desc": np.concatenate([dL_true, C.random_descriptors(r_desc, n_dis)])}
    right = {"x": np.concatenate([xR, (xdr * sf[lv_dis_r]).astype(np.float32)]),
             "y": np.concatenate([yR, (ydr * sf[lv_dis_r]).astype(np.float32)]),
             "octave": np.concatenate([lvR, lv_dis_r]).astype(np.uint8),
             "desc": np.concatenate([dR_true, C.random_descriptors(r_desc, n_dis)])}
    pl = r_kp.permutation(n_kp)
    pr = r_kp.permutation(n_kp)
    left = C.permute_keypoints(left, pl)
    right = C.permute_keypoints(right, pr)
    inv_l = np.argsort(pl)
    inv_r = np.argsort(pr)
    true_pairs = np.stack([inv_l[:n_true], inv_r[:n_true]], axis=1)

    # ---- local map -------------------------------------------------------
    O_true = np.zeros(3)
    n_from = min(n_true, n_map)
    pick = r_map.choice(n_true, n_from, replace=False)
    Z = np.clip(float(cam["bf"]) / np.maximum(d_true[pick], 1e-6), 1.0, 15.0)
    P_kp = back_project(xL[pick].astype(np.float64), yL[pick].astype(np.float64), Z, cam)
    n_uni = n_map - n_from
    P_uni = back_project(r_map.uniform(0, W, n_uni), r_map.uniform(0, H, n_uni),
                         r_map.uniform(1.0, 15.0, n_uni), cam)
    P = np.concatenate([P_kp, P_uni])
    o_ref = np.concatenate([lv_true[pick], r_map.integers(0, C.N_LEVELS, n_uni)])
    mdesc = np.concatenate([C.flip_bits(r_map, dL_true[pick], r_map.integers(0, 25, n_from)),
                            C.random_descriptors(r_map, n_uni)])
    mp = C.map_point_fields(r_map, P, O_true, o_ref, sc, mdesc)
    pm = r_map.permutation(n_map)
    mp = {k: np.ascontiguousarray(v[pm]) for k, v in mp.items()}
    inv_m = np.argsort(pm)
    true_mp = np.stack([inv_m[:n_from], inv_l[pick]], axis=1)

    R_cw, t_cw, O_w = C.perturbed_pose(r_pose, np.eye(3), np.zeros(3))
    pre = (r_pose.random(n_kp) < preassigned_frac).astype(np.uint8)

    frame = {
        "kind": "pinhole",
        "scales": sc,
        "left": left, "right": right,
        "stereo_cam": {"fx": cam["fx"], "bf": cam["bf"], "b": cam["b"], "rows": H},
        "stereo_params": C.pinhole_stereo_params(),
        "map": mp,
        "search": [{
            "cam": {"model": 0, "fx": cam["fx"], "fy": cam["fy"], "cx": cam["cx"],
                    "cy": cam["cy"], "k": np.zeros(4, np.float32), "bf": cam["bf"],
                    "bounds": np.array([0, W, 0, H], np.float32),
                    **C.pose_dict(R_cw, t_cw, O_w)},
            "image": "left",
            "grid": tuple(grid),
            "preassigned": pre,
            "use_u_right": True,
        }],
        "search_params": C.search_params(th),
        "truth": {"stereo_pairs": true_pairs, "map_kp": true_mp, "disparity": d_true},
        "size": {"W": W, "H": H},
    }
    if images:
        frame["pyr_left"] = pyramid(left_img, sc)
        frame["pyr_right"] = pyramid(right_img, sc)
    return frame
