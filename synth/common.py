"""Seeded building blocks for the synthetic workloads.

Nothing here matches, searches or refines anything: these helpers only lay out
scenes (scale tables, ORB-style per-level keypoint budgets, descriptor noise,
rigid poses) so that the oracle and the GPU path can be fed identical bytes.
All geometry here is the scene generator's own float64 arithmetic.
"""
from __future__ import annotations

import numpy as np

N_LEVELS = 8
SCALE_FACTOR = 1.2
DESC_BYTES = 32
MASTER_SEED = 10757000


def f32(v):
    return np.float32(v)


def scale_tables(n_levels: int = N_LEVELS, factor: float = SCALE_FACTOR):
    """Per-level scale tables in binary32 built by repeated multiplication.

    sf[0] = 1, sf[l] = fl32(sf[l-1] * fl32(factor)); inv_sf = fl32(1/sf);
    sigma2 = fl32(sf*sf).  These tables are caller-supplied inputs to both the
    oracle and the device path, so both see the very same bits.
    """
    sf = np.empty(n_levels, np.float32)
    sf[0] = np.float32(1.0)
    fac = np.float32(factor)
    for l in range(1, n_levels):
        sf[l] = np.float32(sf[l - 1] * fac)
    inv_sf = (np.float32(1.0) / sf).astype(np.float32)
    sigma2 = (sf * sf).astype(np.float32)
    return {"sf": sf, "inv_sf": inv_sf, "sigma2": sigma2}


def level_allocation(n: int, n_levels: int = N_LEVELS, factor: float = SCALE_FACTOR):
    """ORB-style geometric split of a keypoint budget over pyramid levels.

    Level l receives round(n * (1-s)/(1-s^L) * s^l) with s = 1/factor; the last
    level takes the remainder.  For n = 1200 this gives
    [261, 217, 181, 151, 126, 105, 87, 72].
    """
    s = 1.0 / factor
    per = n * (1.0 - s) / (1.0 - s ** n_levels)
    out = []
    total = 0
    for _ in range(n_levels - 1):
        k = int(np.floor(per + 0.5))
        out.append(k)
        total += k
        per *= s
    out.append(max(n - total, 0))
    return np.array(out, np.int64)


def random_descriptors(rng, n: int) -> np.ndarray:
    return rng.integers(0, 256, size=(n, DESC_BYTES), dtype=np.uint8)


def flip_bits(rng, desc: np.ndarray, k: np.ndarray) -> np.ndarray:
    """XOR each row of `desc` with k[i] distinct random bit positions."""
    out = desc.copy()
    bits = np.unpackbits(out, axis=1, bitorder="little")
    for i in range(out.shape[0]):
        if k[i] > 0:
            pos = rng.choice(DESC_BYTES * 8, size=int(k[i]), replace=False)
            bits[i, pos] ^= 1
    return np.packbits(bits, axis=1, bitorder="little")


def rodrigues(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    kx = np.array([[0.0, -axis[2], axis[1]],
                   [axis[2], 0.0, -axis[0]],
                   [-axis[1], axis[0], 0.0]])
    return np.eye(3) + np.sin(angle) * kx + (1.0 - np.cos(angle)) * (kx @ kx)


def random_unit(rng, n: int | None = None) -> np.ndarray:
    if n is None:
        v = rng.standard_normal(3)
        return v / np.linalg.norm(v)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def perturbed_pose(rng, R_cw: np.ndarray, t_cw: np.ndarray,
                   trans_m: float = 0.02, rot_deg: float = 0.5):
    """Return (R, t, O) of a pose whose centre moved `trans_m` metres in a random
    direction and whose orientation turned `rot_deg` degrees about a random axis."""
    O = -R_cw.T @ t_cw
    O2 = O + trans_m * random_unit(rng)
    R2 = rodrigues(random_unit(rng), np.deg2rad(rot_deg)) @ R_cw
    t2 = -R2 @ O2
    return R2, t2, O2


def rotate_within(rng, v: np.ndarray, max_deg: float) -> np.ndarray:
    """Rotate each unit row of v by a random angle in [0, max_deg] about a random
    axis perpendicular to it.  The draws are taken row by row (a direction, then
    an angle), the rotation itself is done for all rows at once."""
    n = v.shape[0]
    g = np.empty((n, 3))
    ang = np.empty(n)
    for i in range(n):
        g[i] = rng.standard_normal(3)
        ang[i] = rng.uniform(0.0, max_deg)
    a = g / np.linalg.norm(g, axis=1, keepdims=True)
    a = a - np.sum(a * v, axis=1, keepdims=True) * v
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    th = np.deg2rad(ang)[:, None]
    av = np.cross(a, v)
    # Rodrigues' formula for an axis perpendicular to the vector
    return v + av * np.sin(th) + np.cross(a, av) * (1.0 - np.cos(th))


def pose_dict(R, t, O):
    return {"R": np.asarray(R, np.float32).reshape(3, 3),
            "t": np.asarray(t, np.float32).reshape(3),
            "O": np.asarray(O, np.float32).reshape(3)}


def map_point_fields(rng, P_w: np.ndarray, O_w: np.ndarray, o_ref: np.ndarray,
                     sc: dict, desc: np.ndarray):
    """Map point record: position, viewing normal, distance bounds, descriptor.

    dmax = dist * sf[o_ref] and dmin = dmax / sf[top], which makes the level
    predicted at the reference distance equal o_ref.
    """
    PO = P_w - O_w[None, :]
    dist = np.linalg.norm(PO, axis=1)
    ray = PO / dist[:, None]
    normal = rotate_within(rng, ray, 10.0)
    dmax = dist * sc["sf"][o_ref].astype(np.float64)
    dmin = dmax / float(sc["sf"][-1])
    return {"pos": P_w.astype(np.float32),
            "normal": normal.astype(np.float32),
            "dmin": dmin.astype(np.float32),
            "dmax": dmax.astype(np.float32),
            "desc": np.ascontiguousarray(desc, dtype=np.uint8)}


def permute_keypoints(kp: dict, perm: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(v[perm]) for k, v in kp.items()}


def on_level_grid(v: np.ndarray, level: np.ndarray, sc: dict) -> np.ndarray:
    """Level-0 coordinate of an integer pixel on `level`: fl32(round(v/sf)*sf)."""
    sf = sc["sf"][level].astype(np.float64)
    return (np.rint(v / sf) * sf).astype(np.float32)


def pinhole_stereo_params():
    """Matching constants of the rectified stereo search (values restated from
    the ORB-SLAM3 tracking that the paper accelerates)."""
    return {"th_orb": 75, "half_win": 5, "half_range": 5, "band": 2.0,
            "level_window": 1, "median_num": 21, "median_den": 10}


def fisheye_stereo_params():
    return {"ratio_num": 7, "ratio_den": 10, "cos_parallax_max": 0.9998,
            "chi2": 5.991, "max_theta_deg": 88.0, "newton_iters": 10,
            "newton_tol": 1e-12}


def search_params(th: float = 2.0, level_lo: int = 1, level_hi: int = 1):
    return {"th": th, "view_cos_limit": 0.5, "view_cos_narrow": 0.998,
            "r_narrow": 2.5, "r_wide": 4.0, "dist_lo": 0.8, "dist_hi": 1.2,
            "level_lo": level_lo, "level_hi": level_hi, "th_high": 100,
            "ratio_num": 4, "ratio_den": 5, "ratio_same_level_only": 1}
