"""Seeded fisheye (Kannala-Brandt) stereo frame with its local map.

Shaped like a TUM-VI frame: 512x512 per camera, fx = fy = 190, per-camera
k1..k4 ~ U[-0.01, 0.01], the right camera 0.10 m along the left x axis and
turned 2 degrees about y.  Keypoints are projections of seeded 3D points
(ray angle <= 75 degrees, 1-15 m) rounded on their pyramid level plus 20%
distractors.  There are no images: fisheye stereo has no patch refinement.
"""
from __future__ import annotations

import numpy as np

from . import common as C
from .images import level_sizes

BORDER = 16


def kb_camera(rng, W=512, H=512, f=190.0, kmax=0.01):
    return {"W": W, "H": H, "fx": np.float32(f), "fy": np.float32(f),
            "cx": np.float32(W / 2), "cy": np.float32(H / 2),
            "k": rng.uniform(-kmax, kmax, 4).astype(np.float32)}


def kb_project64(X: np.ndarray, cam: dict) -> np.ndarray:
    """Scene-generator projection (float64): theta_d = theta*(1+k1 t^2+...+k4 t^8)."""
    k = cam["k"].astype(np.float64)
    rho = np.hypot(X[:, 0], X[:, 1])
    th = np.arctan2(rho, X[:, 2])
    t2 = th * th
    thd = th * (1 + k[0] * t2 + k[1] * t2 ** 2 + k[2] * t2 ** 3 + k[3] * t2 ** 4)
    s = np.where(rho > 0, thd / np.where(rho > 0, rho, 1.0), 0.0)
    u = float(cam["fx"]) * X[:, 0] * s + float(cam["cx"])
    v = float(cam["fy"]) * X[:, 1] * s + float(cam["cy"])
    return np.stack([u, v], axis=1)


def cap_directions(rng, n, max_deg=75.0):
    cmin = np.cos(np.deg2rad(max_deg))
    c = rng.uniform(cmin, 1.0, n)
    s = np.sqrt(1 - c * c)
    phi = rng.uniform(0, 2 * np.pi, n)
    return np.stack([s * np.cos(phi), s * np.sin(phi), c], axis=1)


def _theta(X):
    return np.arctan2(np.hypot(X[:, 0], X[:, 1]), X[:, 2])


def fisheye_frame(seed, n_kp: int = 1500, n_map: int = 5000, grid=(64, 48),
                  th: float = 2.0, preassigned_frac: float = 0.1,
                  baseline: float = 0.10, rot_deg: float = 2.0,
                  overlap_frac: float = 0.6):
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    r_cam, r_kp, r_desc, r_map, r_pose = [np.random.default_rng(s) for s in ss.spawn(5)]
    camL = kb_camera(r_cam)
    camR = kb_camera(r_cam)
    W, H = camL["W"], camL["H"]
    sc = C.scale_tables()
    sf = sc["sf"].astype(np.float64)
    ws, hs = level_sizes(W, H, sc)

    R_lr = C.rodrigues(np.array([0.0, 1.0, 0.0]), np.deg2rad(rot_deg))
    t_lr = np.array([baseline, 0.0, 0.0])
    R_rl = R_lr.T
    t_rl = -R_lr.T @ t_lr

    alloc_l = np.repeat(np.arange(C.N_LEVELS), C.level_allocation(n_kp))
    r_kp.shuffle(alloc_l)
    n_true = int(round(0.8 * n_kp))
    lv_true = alloc_l[:n_true]

    XL = np.zeros((n_true, 3))
    uvL = np.zeros((n_true, 2), np.float32)
    uvR = np.zeros((n_true, 2), np.float32)
    lvR = np.zeros(n_true, np.int64)
    todo = np.arange(n_true)
    for _ in range(500):
        if todo.size == 0:
            break
        m = todo.size
        X = cap_directions(r_kp, m) * r_kp.uniform(1.0, 15.0, m)[:, None]
        Xr = X @ R_rl.T + t_rl
        l = lv_true[todo]
        same = r_kp.random(m) < 0.85
        step = np.where(r_kp.random(m) < 0.5, -1, 1)
        lr = np.where(same, l, np.clip(l + step, 0, C.N_LEVELS - 1))
        pl = kb_project64(X, camL)
        pr = kb_project64(Xr, camR)
        ql = np.rint(pl / sf[l][:, None])
        qr = np.rint(pr / sf[lr][:, None])
        wl = np.array([ws[k] for k in l]); hl = np.array([hs[k] for k in l])
        wr = np.array([ws[k] for k in lr]); hr = np.array([hs[k] for k in lr])
        ok = ((Xr[:, 2] > 0) & (_theta(Xr) < np.deg2rad(75.0)) &
              (ql[:, 0] >= BORDER) & (ql[:, 0] < wl - BORDER) &
              (ql[:, 1] >= BORDER) & (ql[:, 1] < hl - BORDER) &
              (qr[:, 0] >= BORDER) & (qr[:, 0] < wr - BORDER) &
              (qr[:, 1] >= BORDER) & (qr[:, 1] < hr - BORDER))
        idx = todo[ok]
        XL[idx] = X[ok]
        uvL[idx] = (ql[ok] * sf[l[ok]][:, None]).astype(np.float32)
        uvR[idx] = (qr[ok] * sf[lr[ok]][:, None]).astype(np.float32)
        lvR[idx] = lr[ok]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("could not place fisheye pairs")

    base = C.random_descriptors(r_desc, n_true)
    dR = C.flip_bits(r_desc, base, r_desc.integers(0, 25, n_true))
    n_dis = n_kp - n_true

    def distractors(levels):
        x = np.array([r_kp.integers(BORDER, ws[l] - BORDER) for l in levels]) * sf[levels]
        y = np.array([r_kp.integers(BORDER, hs[l] - BORDER) for l in levels]) * sf[levels]
        return x.astype(np.float32), y.astype(np.float32)

    lv_dl = alloc_l[n_true:]
    alloc_r = np.repeat(np.arange(C.N_LEVELS), C.level_allocation(n_kp))
    r_kp.shuffle(alloc_r)
    lv_dr = alloc_r[:n_dis]
    xdl, ydl = distractors(lv_dl)
    xdr, ydr = distractors(lv_dr)
    left = {"x": np.concatenate([uvL[:, 0], xdl]), "y": np.concatenate([uvL[:, 1], ydl]),
            "octave": np.concatenate([lv_true, lv_dl]).astype(np.uint8),
            "desc": np.concatenate([base, C.random_descriptors(r_desc, n_dis)])}
    right = {"x": np.concatenate([uvR[:, 0], xdr]), "y": np.concatenate([uvR[:, 1], ydr]),
             "octave": np.concatenate([lvR, lv_dr]).astype(np.uint8),
             "desc": np.concatenate([dR, C.random_descriptors(r_desc, n_dis)])}
    pl_ = r_kp.permutation(n_kp)
    pr_ = r_kp.permutation(n_kp)
    left = C.permute_keypoints(left, pl_)
    right = C.permute_keypoints(right, pr_)
    inv_l = np.argsort(pl_)
    inv_r = np.argsort(pr_)
    true_pairs = np.stack([inv_l[:n_true], inv_r[:n_true]], axis=1)

    # ---- local map (points behind true keypoints + uniform extras) --------
    n_from = min(n_true, n_map)
    pick = r_map.choice(n_true, n_from, replace=False)
    n_uni = n_map - n_from
    X_uni = cap_directions(r_map, n_uni) * r_map.uniform(1.0, 15.0, n_uni)[:, None]
    P = np.concatenate([XL[pick], X_uni])
    o_ref = np.concatenate([lv_true[pick], r_map.integers(0, C.N_LEVELS, n_uni)])
    mdesc = np.concatenate([C.flip_bits(r_map, base[pick], r_map.integers(0, 25, n_from)),
                            C.random_descriptors(r_map, n_uni)])
    mp = C.map_point_fields(r_map, P, np.zeros(3), o_ref, sc, mdesc)
    pm = r_map.permutation(n_map)
    mp = {k: np.ascontiguousarray(v[pm]) for k, v in mp.items()}
    inv_m = np.argsort(pm)

    R_lw, t_lw, O_l = C.perturbed_pose(r_pose, np.eye(3), np.zeros(3))
    R_rw = R_rl @ R_lw
    t_rw = R_rl @ t_lw + t_rl
    O_r = -R_rw.T @ t_rw

    def search_cam(cam, R, t, O):
        return {"model": 1, "fx": cam["fx"], "fy": cam["fy"], "cx": cam["cx"],
                "cy": cam["cy"], "k": cam["k"], "bf": np.float32(0.0),
                "bounds": np.array([0, W, 0, H], np.float32), **C.pose_dict(R, t, O)}

    a_l = np.float32((1.0 - overlap_frac) * W)
    b_r = np.float32(overlap_frac * W)
    frame = {
        "kind": "fisheye",
        "scales": sc,
        "left": left, "right": right,
        "stereo_cam": {
            "left": {k: camL[k] for k in ("fx", "fy", "cx", "cy", "k")},
            "right": {k: camR[k] for k in ("fx", "fy", "cx", "cy", "k")},
            "R_lr": R_lr.astype(np.float32), "t_lr": t_lr.astype(np.float32),
            "overlap_left": np.array([a_l, np.float32(W)], np.float32),
            "overlap_right": np.array([0.0, b_r], np.float32),
        },
        "stereo_params": C.fisheye_stereo_params(),
        "map": mp,
        "search": [
            {"cam": search_cam(camL, R_lw, t_lw, O_l), "image": "left", "grid": tuple(grid),
             "preassigned": (r_pose.random(n_kp) < preassigned_frac).astype(np.uint8),
             "use_u_right": False},
            {"cam": search_cam(camR, R_rw, t_rw, O_r), "image": "right", "grid": tuple(grid),
             "preassigned": (r_pose.random(n_kp) < preassigned_frac).astype(np.uint8),
             "use_u_right": False},
        ],
        "search_params": C.search_params(th),
        "truth": {"stereo_pairs": true_pairs, "points": XL,
                  "map_kp": np.stack([inv_m[:n_from], inv_l[pick]], axis=1)},
        "size": {"W": W, "H": H},
    }
    return frame
