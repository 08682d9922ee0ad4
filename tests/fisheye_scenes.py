"""Hand-built fisheye stereo scenes that decide one test of the triangulation
check each (parallax, depth in either camera, reprojection in either view),
with the expected outcome of every pair computed by an independent route:

  - rays: the Kannala-Brandt radius equation solved by bracketing (scipy
    brentq) instead of Newton's method;
  - the point: numpy least squares (SVD) on the linear two-view system
    instead of Cramer's rule on its normal equations;
  - projections: the scene generator's own float64 projector.

Keypoint pairs share one descriptor (distance 0) and every other descriptor is
random, so every pair passes the nearest-neighbour and ratio stages and only
the geometric tests decide.  Expected outcomes are kept only where every tested
quantity lies at least `margin` (relative) away from its threshold, so the two
numerical routes cannot disagree on a decision.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

import synth
from synth.fisheye import kb_project64

f32 = np.float32


def unproject(cam, u, v):
    """Unit-z ray of pixel (u, v) (float64), or None beyond 89 degrees."""
    k = np.asarray(cam["k"], np.float64)
    xp = (float(u) - float(cam["cx"])) / float(cam["fx"])
    yp = (float(v) - float(cam["cy"])) / float(cam["fy"])
    r = np.hypot(xp, yp)
    if r < 1e-12:
        return np.array([xp, yp, 1.0])
    f = lambda th: th * (1 + k[0] * th ** 2 + k[1] * th ** 4 + k[2] * th ** 6 + k[3] * th ** 8) - r
    # bracket on the increasing branch of the radius curve (with |k| ~ 0.01 it
    # may turn over below 89 degrees)
    grid = np.linspace(0.0, np.deg2rad(89.0), 8901)
    vals = f(grid)
    top = int(np.argmax(vals))
    lim = grid[top]
    if vals[top] < 0:
        return None
    th = brentq(f, 0.0, lim, xtol=1e-15, rtol=1e-15)
    s = np.tan(th) / r
    return np.array([xp * s, yp * s, 1.0])


def lstsq_point(r1, r2, R_lr, t_lr):
    """Linear two-view triangulation (homogeneous coordinate fixed to 1), left
    camera [I|0], right camera [R_lr^T | -R_lr^T t_lr], solved by SVD."""
    R = np.asarray(R_lr, np.float64)
    t = np.asarray(t_lr, np.float64)
    Rrl, trl = R.T, -R.T @ t
    p1, p2 = r1[:2] / r1[2], r2[:2] / r2[2]
    A = np.array([[-1.0, 0.0, p1[0]], [0.0, -1.0, p1[1]],
                  p2[0] * Rrl[2] - Rrl[0], p2[1] * Rrl[2] - Rrl[1]])
    b = np.array([0.0, 0.0, -(p2[0] * trl[2] - trl[0]), -(p2[1] * trl[2] - trl[1])])
    return np.linalg.lstsq(A, b, rcond=None)[0]


def expected_pair(cam, sc, sp, uL, uR, oL, oR, margin=0.01):
    """Outcome of the triangulation check for one pair: (accepted, reason,
    clear) where reason names the first failing test and clear says that no
    tested quantity lies within `margin` of its threshold."""
    R = cam["R_lr"].astype(np.float64)
    t = cam["t_lr"].astype(np.float64)
    r1 = unproject(cam["left"], *uL)
    r2 = unproject(cam["right"], *uR)
    if r1 is None or r2 is None:
        return False, "theta", False
    th_max = np.deg2rad(sp["max_theta_deg"])
    th1 = np.arctan(np.hypot(r1[0], r1[1]))
    th2 = np.arctan(np.hypot(r2[0], r2[1]))
    clear = abs(th1 - th_max) > 1e-3 and abs(th2 - th_max) > 1e-3
    if th1 >= th_max or th2 >= th_max:
        return False, "theta", clear
    r21 = R @ r2
    cosp = r1 @ r21 / (np.linalg.norm(r1) * np.linalg.norm(r21))
    cmax = sp["cos_parallax_max"]
    clear = clear and abs(cosp - cmax) > margin * (1 - cmax)
    if cosp > cmax:
        return False, "parallax", clear
    X = lstsq_point(r1, r2, R, t)
    X2 = R.T @ (X - t)
    clear = clear and abs(X[2]) > 1e-6 and abs(X2[2]) > 1e-6
    if X[2] <= 0 or X2[2] <= 0:
        return False, "depth", clear
    s2 = sc["sigma2"].astype(np.float64)
    eL = ((kb_project64(X[None], cam["left"])[0] - np.asarray(uL, np.float64)) ** 2).sum()
    eR = ((kb_project64(X2[None], cam["right"])[0] - np.asarray(uR, np.float64)) ** 2).sum()
    gL, gR = sp["chi2"] * s2[oL], sp["chi2"] * s2[oR]
    clear = clear and abs(eL - gL) > margin * gL and abs(eR - gR) > margin * gR
    if eL > gL or eR > gR:
        return False, "reproj", clear
    return True, "ok", clear


def _base(seed):
    f = synth.tiny_fisheye(seed, n_kp=40)
    W = f["size"]["W"]
    f["stereo_cam"] = dict(f["stereo_cam"])
    f["stereo_cam"]["overlap_left"] = np.array([0, W], np.float32)
    f["stereo_cam"]["overlap_right"] = np.array([0, W], np.float32)
    f["stereo_params"] = dict(f["stereo_params"])
    return f


def _install(f, uvL, uvR, oL, oR, rng):
    n = len(uvL)
    desc = rng.integers(0, 256, (n, 32), dtype=np.uint8)
    f["left"] = {"x": uvL[:, 0].astype(np.float32), "y": uvL[:, 1].astype(np.float32),
                 "octave": np.asarray(oL, np.uint8), "desc": desc}
    f["right"] = {"x": uvR[:, 0].astype(np.float32), "y": uvR[:, 1].astype(np.float32),
                  "octave": np.asarray(oR, np.uint8), "desc": desc.copy()}
    f["search"] = [dict(s) for s in f["search"]]
    for s in f["search"]:
        s["preassigned"] = np.zeros(n, np.uint8)
    f.pop("truth", None)
    return f


def _inside(uv, W):
    return (uv >= 1).all(1) & (uv <= W - 1).all(1)


def parallax_scene(seed=91):
    """Noise-free pairs whose rays meet at angles whose cosine is spread tightly
    around the parallax limit (level 0, so the reprojection gate is tight
    too)."""
    f = _base(seed)
    rng = np.random.default_rng(seed)
    cam = f["stereo_cam"]
    R = cam["R_lr"].astype(np.float64)
    t = cam["t_lr"].astype(np.float64)
    cmax = f["stereo_params"]["cos_parallax_max"]
    gaps = np.array([-3e-5, -1e-5, -4e-6, -2e-6, 2e-6, 4e-6, 1e-5, 3e-5, 1e-4])
    uvL, uvR = [], []
    while len(uvL) < 3 * len(gaps):
        for g in gaps:
            d = synth.fisheye.cap_directions(rng, 1, 55.0)[0]

            def cosp(s, d=d):
                X = d * s
                return X @ (X - t) / (np.linalg.norm(X) * np.linalg.norm(X - t)) - (cmax + g)
            if cosp(0.5) > 0 or cosp(500.0) < 0:
                continue
            X = d * brentq(cosp, 0.5, 500.0, xtol=1e-12)
            pl = kb_project64(X[None], cam["left"])
            pr = kb_project64((R.T @ (X - t))[None], cam["right"])
            if not (_inside(pl, 512)[0] and _inside(pr, 512)[0]):
                continue
            uvL.append(pl[0]); uvR.append(pr[0])
    uvL = np.array(uvL, np.float32); uvR = np.array(uvR, np.float32)
    n = len(uvL)
    return _install(f, uvL, uvR, np.zeros(n), np.zeros(n), rng)


def depth_scene(seed=92):
    """Pairs whose lines meet behind the right camera (in front of the left)
    or behind the left camera (in front of the right), beside pairs in front
    of both; the right camera is turned 30 degrees so that such points are
    seen within 80 degrees of both axes, and the reprojection gate is opened
    (chi2 = 1e12) so that the depth tests alone decide."""
    f = _base(seed)
    rng = np.random.default_rng(seed)
    cam = f["stereo_cam"]
    R = synth.common.rodrigues(np.array([0.0, 1.0, 0.0]), np.deg2rad(-30.0))
    t = np.array([0.1, 0.0, 0.0])
    cam["R_lr"] = R.astype(np.float32)
    cam["t_lr"] = t.astype(np.float32)
    R = cam["R_lr"].astype(np.float64)
    t = cam["t_lr"].astype(np.float64)
    f["stereo_params"]["chi2"] = 1e12
    lim = np.deg2rad(80.0)

    def th(X):
        return np.arctan2(np.hypot(X[0], X[1]), X[2])
    want = {"front": 8, "behind_right": 8, "behind_left": 8}
    got = {k: [] for k in want}
    for _ in range(200000):
        if all(len(got[k]) >= want[k] for k in want):
            break
        X = rng.uniform(-4, 4, 3)
        X2 = R.T @ (X - t)
        # the keypoint of a camera that has the point behind it lies on the
        # line's other half (antipodal direction)
        a = X if X[2] > 0 else -X
        b = X2 if X2[2] > 0 else -X2
        if th(a) > lim or th(b) > lim or np.linalg.norm(X) < 0.3:
            continue
        kind = ("front" if X[2] > 0 and X2[2] > 0 else "behind_right" if X[2] > 0 else
                "behind_left" if X2[2] > 0 else None)
        if kind is None or len(got[kind]) >= want[kind]:
            continue
        pl = kb_project64(a[None], cam["left"])
        pr = kb_project64(b[None], cam["right"])
        if not (_inside(pl, 512)[0] and _inside(pr, 512)[0]):
            continue
        got[kind].append((pl[0], pr[0]))
    pairs = got["front"] + got["behind_right"] + got["behind_left"]
    uvL = np.array([p[0] for p in pairs], np.float32)
    uvR = np.array([p[1] for p in pairs], np.float32)
    n = len(pairs)
    return _install(f, uvL, uvR, np.zeros(n), np.zeros(n), rng)


def reprojection_scene(seed=93):
    """Pairs whose right keypoint is moved 0.5-14 px off the exact projection,
    the two keypoints on different pyramid levels (one view's gate 12.8x the
    other's), so that the reprojection test of each view, with its own
    keypoint's level, decides."""
    f = _base(seed)
    rng = np.random.default_rng(seed)
    cam = f["stereo_cam"]
    R = cam["R_lr"].astype(np.float64)
    t = cam["t_lr"].astype(np.float64)
    uvL, uvR, oL, oR = [], [], [], []
    while len(uvL) < 160:
        X = synth.fisheye.cap_directions(rng, 1, 50.0)[0] * rng.uniform(1.5, 4.0)
        pl = kb_project64(X[None], cam["left"])
        pr = kb_project64((R.T @ (X - t))[None], cam["right"])
        ang = rng.uniform(0, 2 * np.pi)
        pr = pr + rng.uniform(0.5, 14.0) * np.array([[np.cos(ang), np.sin(ang)]])
        if not (_inside(pl, 512)[0] and _inside(pr, 512)[0]):
            continue
        uvL.append(pl[0]); uvR.append(pr[0])
        lo, hi = (7, int(rng.integers(0, 3))) if len(uvL) % 2 else (int(rng.integers(0, 3)), 7)
        oL.append(lo); oR.append(hi)
    return _install(f, np.array(uvL, np.float32), np.array(uvR, np.float32), oL, oR, rng)


def expected(f):
    """(accepted, reason, clear) per left keypoint i (paired with right i)."""
    L, R = f["left"], f["right"]
    out = []
    for i in range(len(L["x"])):
        out.append(expected_pair(f["stereo_cam"], f["scales"], f["stereo_params"],
                                 (L["x"][i], L["y"][i]), (R["x"][i], R["y"][i]),
                                 int(L["octave"][i]), int(R["octave"][i])))
    return out
