"""Seeded multi-stream serving workload.

A world of seeded 3D points (uniform + Gaussian blobs in a 200 x 200 x 20 m
box); camera streams of either kind (rectified pinhole 752x480 or
Kannala-Brandt fisheye 512x512) moving along smooth 6-DoF trajectories (two
sinusoids per axis, mean speed 0.5-2 m/s, looking along the velocity with a
small roll and pitch); each stream keeps a local map of its N_s nearest world
points (N_s ~ U[2000, 40000]); frames arrive as a Poisson process at a
per-stream rate of 20-30 Hz.  Frames are pre-generated into a small pool per
stream (keypoints are projections of visible map points plus 20% distractors)
and cycled; pinhole image pyramids come from a shared pool, since image content
does not change the amount of work.

With `map_churn` > 0 a stream's local map changes from frame to frame, as
Update Local Map's output does while the camera moves: before pooled frame q
(q >= 1) a fraction `map_churn` of the map's points leave it and as many
points, not yet in it, join; before the pool starts over, the map returns to
the set it started from.  Edits are given as point ids of the stream's point
table (which slot a point occupies is up to the consumer), and each frame's
keypoints are generated from the points of its own map.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import common as C
from .fisheye import kb_camera, kb_project64
from .images import DisparityField, noise_texture, pyramid, right_image
from .pinhole import pinhole_camera

WORLD_BOX = np.array([200.0, 200.0, 20.0])


def make_world(rng, n_points: int = 2_000_000, n_blobs: int = 2000, blob_frac: float = 0.5):
    n_blob = int(n_points * blob_frac)
    uni = rng.uniform(0, 1, (n_points - n_blob, 3)) * WORLD_BOX
    centres = rng.uniform(0, 1, (n_blobs, 3)) * WORLD_BOX
    which = rng.integers(0, n_blobs, n_blob)
    blob = centres[which] + rng.normal(0, 1.0, (n_blob, 3))
    P = np.concatenate([uni, blob]).astype(np.float64)
    return {"pos": P, "desc": C.random_descriptors(rng, n_points), "tree": cKDTree(P)}


class Trajectory:
    """Sum of two sinusoids per axis around a start point, scaled to a mean speed."""

    def __init__(self, rng, speed: float):
        self.c = rng.uniform([30, 30, 5], [170, 170, 15])
        self.a = rng.uniform(0.5, 1.0, (2, 3)) * np.array([1.0, 1.0, 0.2])
        self.w = rng.uniform(0.1, 0.6, (2, 3))
        self.ph = rng.uniform(0, 2 * np.pi, (2, 3))
        ts = np.linspace(0, 20, 2001)
        v = np.linalg.norm(np.gradient(self._raw(ts), ts, axis=0), axis=1).mean()
        self.scale = speed / max(v, 1e-9)
        self.roll = rng.uniform(-0.05, 0.05)

    def _raw(self, t):
        t = np.atleast_1d(t)[:, None, None]
        return (self.a[None] * np.sin(self.w[None] * t + self.ph[None])).sum(1)

    def position(self, t):
        return self.c + self.scale * self._raw(t)[0]

    def pose(self, t, dt=1e-3):
        """World-to-camera (R, t, O): camera z along the velocity."""
        O = self.position(t)
        vel = (self.position(t + dt) - self.position(t - dt)) / (2 * dt)
        z = vel / max(np.linalg.norm(vel), 1e-9)
        up = np.array([0.0, 0.0, 1.0])
        x = np.cross(up, z)
        x /= max(np.linalg.norm(x), 1e-9)
        y = np.cross(z, x)
        Rwc = np.stack([x, y, z], axis=1)          # columns: camera axes in the world
        Rwc = Rwc @ C.rodrigues(np.array([0.0, 0.0, 1.0]), self.roll)
        R = Rwc.T
        return R, -R @ O, O


def _stream_map(rng, world, centre, n, sc):
    _, idx = world["tree"].query(centre, k=n)
    P = world["pos"][idx]
    o_ref = rng.integers(0, C.N_LEVELS, n)
    mp = C.map_point_fields(rng, P, centre, o_ref, sc, world["desc"][idx])
    return mp, P, o_ref


def _kp_levels(P, O, dmax, sf, rng):
    dist = np.linalg.norm(P - O, axis=1)
    ratio = dmax / np.maximum(dist, 1e-9)
    pred = np.searchsorted(sf.astype(np.float64), ratio)
    pred = np.clip(pred, 0, C.N_LEVELS - 1)
    return np.clip(pred + rng.integers(-1, 2, len(P)), 0, C.N_LEVELS - 1)


def _pinhole_frame_kps(rng, mp, P, cam, R, t, O, n_kp, sc):
    W, H = cam["W"], cam["H"]
    sf = sc["sf"].astype(np.float64)
    Pc = P @ R.T + t
    z = Pc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = float(cam["fx"]) * Pc[:, 0] / z + float(cam["cx"])
        v = float(cam["fy"]) * Pc[:, 1] / z + float(cam["cy"])
    d = float(cam["bf"]) / np.where(z > 0, z, 1.0)
    ok = (z > 0.5) & (u >= 20) & (u < W - 20) & (v >= 20) & (v < H - 20) & (u - d >= 20)
    vis = np.nonzero(ok)[0]
    n_true = min(len(vis), int(round(0.8 * n_kp)))
    pick = rng.choice(vis, n_true, replace=False) if n_true else np.zeros(0, np.int64)
    lv = _kp_levels(P[pick], O, mp["dmax"][pick].astype(np.float64), sc["sf"], rng)
    xl = (np.rint(u[pick] / sf[lv]) * sf[lv]).astype(np.float32)
    yl = (np.rint(v[pick] / sf[lv]) * sf[lv]).astype(np.float32)
    xr = (np.rint((u[pick] - d[pick]) / sf[lv]) * sf[lv]).astype(np.float32)
    yr = ((np.rint(v[pick] / sf[lv]) + rng.integers(-1, 2, n_true)) * sf[lv]).astype(np.float32)
    base = mp["desc"][pick]
    dl = C.flip_bits(rng, base, rng.integers(0, 25, n_true))
    dr = C.flip_bits(rng, base, rng.integers(0, 25, n_true))
    n_dis = n_kp - n_true

    def distract():
        lvd = rng.integers(0, C.N_LEVELS, n_dis)
        return (np.rint(rng.uniform(20, W - 20, n_dis) / sf[lvd]) * sf[lvd]).astype(np.float32), \
               (np.rint(rng.uniform(20, H - 20, n_dis) / sf[lvd]) * sf[lvd]).astype(np.float32), lvd
    xdl, ydl, lvl_ = distract()
    xdr, ydr, lvr_ = distract()
    left = {"x": np.concatenate([xl, xdl]), "y": np.concatenate([yl, ydl]),
            "octave": np.concatenate([lv, lvl_]).astype(np.uint8),
            "desc": np.concatenate([dl, C.random_descriptors(rng, n_dis)])}
    right = {"x": np.concatenate([xr, xdr]), "y": np.concatenate([yr, ydr]),
             "octave": np.concatenate([lv, lvr_]).astype(np.uint8),
             "desc": np.concatenate([dr, C.random_descriptors(rng, n_dis)])}
    return C.permute_keypoints(left, rng.permutation(n_kp)), C.permute_keypoints(right, rng.permutation(n_kp))


def _fisheye_frame_kps(rng, mp, P, camL, camR, R_rl, t_rl, R, t, O, n_kp, sc):
    sf = sc["sf"].astype(np.float64)
    Pc = P @ R.T + t
    Pr = Pc @ R_rl.T + t_rl
    th = np.arctan2(np.hypot(Pc[:, 0], Pc[:, 1]), Pc[:, 2])
    thr = np.arctan2(np.hypot(Pr[:, 0], Pr[:, 1]), Pr[:, 2])
    uvl = kb_project64(Pc, camL)
    uvr = kb_project64(Pr, camR)
    ok = ((th < np.deg2rad(75)) & (thr < np.deg2rad(75)) & (Pc[:, 2] > 0.3) &
          (uvl[:, 0] >= 20) & (uvl[:, 0] < 492) & (uvl[:, 1] >= 20) & (uvl[:, 1] < 492) &
          (uvr[:, 0] >= 20) & (uvr[:, 0] < 492) & (uvr[:, 1] >= 20) & (uvr[:, 1] < 492))
    vis = np.nonzero(ok)[0]
    n_true = min(len(vis), int(round(0.8 * n_kp)))
    pick = rng.choice(vis, n_true, replace=False) if n_true else np.zeros(0, np.int64)
    lv = _kp_levels(P[pick], O, mp["dmax"][pick].astype(np.float64), sc["sf"], rng)
    ql = (np.rint(uvl[pick] / sf[lv][:, None]) * sf[lv][:, None]).astype(np.float32)
    qr = (np.rint(uvr[pick] / sf[lv][:, None]) * sf[lv][:, None]).astype(np.float32)
    base = mp["desc"][pick]
    dl = C.flip_bits(rng, base, rng.integers(0, 25, n_true))
    dr = C.flip_bits(rng, base, rng.integers(0, 25, n_true))
    n_dis = n_kp - n_true

    def distract():
        lvd = rng.integers(0, C.N_LEVELS, n_dis)
        return (np.rint(rng.uniform(20, 492, (n_dis, 2)) / sf[lvd][:, None]) * sf[lvd][:, None]).astype(np.float32), lvd
    qdl, lvl_ = distract()
    qdr, lvr_ = distract()
    left = {"x": np.concatenate([ql[:, 0], qdl[:, 0]]), "y": np.concatenate([ql[:, 1], qdl[:, 1]]),
            "octave": np.concatenate([lv, lvl_]).astype(np.uint8),
            "desc": np.concatenate([dl, C.random_descriptors(rng, n_dis)])}
    right = {"x": np.concatenate([qr[:, 0], qdr[:, 0]]), "y": np.concatenate([qr[:, 1], qdr[:, 1]]),
             "octave": np.concatenate([lv, lvr_]).astype(np.uint8),
             "desc": np.concatenate([dr, C.random_descriptors(rng, n_dis)])}
    return C.permute_keypoints(left, rng.permutation(n_kp)), C.permute_keypoints(right, rng.permutation(n_kp))


def _churn(rng, n_map: int, n_frames: int, k: int):
    """Point-id sets of a map that loses k random points and gains k new ones
    before every frame after the first: (sets, edits), where edits[q] turns
    set q-1 into set q and edits[0] turns the last set back into the first."""
    sets = [np.arange(n_map)]
    edits = [None]
    nxt = n_map
    for _ in range(1, n_frames):
        rem = np.sort(rng.choice(sets[-1], k, replace=False))
        ins = np.arange(nxt, nxt + k)
        nxt += k
        sets.append(np.sort(np.concatenate([np.setdiff1d(sets[-1], rem), ins])))
        edits.append({"remove_ids": rem, "insert_ids": ins})
    edits[0] = {"remove_ids": np.setdiff1d(sets[-1], sets[0]), "insert_ids": np.setdiff1d(sets[0], sets[-1])}
    return sets, edits


def make_streams(seed=None, n_streams: int = 32, frames_per_stream: int = 8,
                 world_points: int = 2_000_000, map_range=(2000, 40000), kp_range=(800, 2000),
                 pyramid_pool: int = 4, rate_range=(20.0, 30.0), map_churn: float = 0.0):
    """Streams, each with a resident map and a pool of frames (synth frame
    dicts).  Without churn every frame shares the stream's map arrays; with
    churn a stream also carries its point table ("points"), the ids of its
    first map ("map_ids0", the order it is uploaded in) and the per-frame
    edits ("edits"), and frame q's "map" holds the points of its map in id
    order (the set, not a slot order)."""
    ss = seed if seed is not None else np.random.SeedSequence(C.MASTER_SEED + 5)
    ctl, wss, pss, *stream_ss = ss.spawn(3 + n_streams)
    rng = np.random.default_rng(ctl)
    world = make_world(np.random.default_rng(wss), world_points)
    sc = C.scale_tables()
    pinhole_cam = pinhole_camera()
    prng = np.random.default_rng(pss)
    pyrs = []
    for _ in range(pyramid_pool):
        left = noise_texture(prng, pinhole_cam["H"], pinhole_cam["W"])
        field = DisparityField(prng, pinhole_cam["W"], pinhole_cam["H"])
        pyrs.append((pyramid(left, sc), pyramid(right_image(prng, left, field), sc)))
    kinds = np.array(["pinhole"] * (n_streams // 2) + ["fisheye"] * (n_streams - n_streams // 2))
    rng.shuffle(kinds)
    streams = []
    for s in range(n_streams):
        r = np.random.default_rng(stream_ss[s])
        traj = Trajectory(r, speed=r.uniform(0.5, 2.0))
        rate = r.uniform(*rate_range)
        n_map = int(r.integers(map_range[0], map_range[1] + 1))
        n_kp = int(r.integers(kp_range[0], kp_range[1] + 1))
        k_churn = int(round(map_churn * n_map)) if frames_per_stream > 1 else 0
        table, P_all, _ = _stream_map(r, world, traj.position(0.0), n_map + k_churn * (frames_per_stream - 1), sc)
        if k_churn:
            id_sets, edits = _churn(r, n_map, frames_per_stream, k_churn)
        else:
            id_sets, edits = [np.arange(n_map)] * frames_per_stream, None
        frames = []
        if kinds[s] == "fisheye":
            camL, camR = kb_camera(r), kb_camera(r)
            R_lr = C.rodrigues(np.array([0.0, 1.0, 0.0]), np.deg2rad(2.0))
            t_lr = np.array([0.10, 0.0, 0.0])
            R_rl, t_rl = R_lr.T, -R_lr.T @ t_lr
        for f in range(frames_per_stream):
            if edits is None:
                mp, P = table, P_all
            else:
                mp = {key: v[id_sets[f]] for key, v in table.items()}
                P = P_all[id_sets[f]]
            tt = f / rate
            R, t, O = traj.pose(tt)
            Rs, ts, Os = C.perturbed_pose(r, R, t)
            pre = (r.random(n_kp) < 0.1).astype(np.uint8)
            if kinds[s] == "pinhole":
                left, right = _pinhole_frame_kps(r, mp, P, pinhole_cam, R, t, O, n_kp, sc)
                pl, pr = pyrs[(s + f) % len(pyrs)]
                cam = pinhole_cam
                frame = {
                    "kind": "pinhole", "scales": sc, "left": left, "right": right,
                    "pyr_left": pl, "pyr_right": pr,
                    "stereo_cam": {"fx": cam["fx"], "bf": cam["bf"], "b": cam["b"], "rows": cam["H"]},
                    "stereo_params": C.pinhole_stereo_params(), "map": mp,
                    "search": [{"cam": {"model": 0, "fx": cam["fx"], "fy": cam["fy"], "cx": cam["cx"],
                                        "cy": cam["cy"], "k": np.zeros(4, np.float32), "bf": cam["bf"],
                                        "bounds": np.array([0, cam["W"], 0, cam["H"]], np.float32),
                                        **C.pose_dict(Rs, ts, Os)},
                                "image": "left", "grid": (64, 48), "preassigned": pre,
                                "use_u_right": True}],
                    "search_params": C.search_params(2.0),
                }
            else:
                left, right = _fisheye_frame_kps(r, mp, P, camL, camR, R_rl, t_rl, R, t, O, n_kp, sc)
                Rr = R_rl @ Rs
                tr = R_rl @ ts + t_rl

                def scam(cam, RR, TT):
                    return {"model": 1, "fx": cam["fx"], "fy": cam["fy"], "cx": cam["cx"], "cy": cam["cy"],
                            "k": cam["k"], "bf": np.float32(0.0),
                            "bounds": np.array([0, 512, 0, 512], np.float32),
                            **C.pose_dict(RR, TT, -RR.T @ TT)}
                frame = {
                    "kind": "fisheye", "scales": sc, "left": left, "right": right,
                    "stereo_cam": {"left": {k: camL[k] for k in ("fx", "fy", "cx", "cy", "k")},
                                   "right": {k: camR[k] for k in ("fx", "fy", "cx", "cy", "k")},
                                   "R_lr": R_lr.astype(np.float32), "t_lr": t_lr.astype(np.float32),
                                   "overlap_left": np.array([0.4 * 512, 512], np.float32),
                                   "overlap_right": np.array([0.0, 0.6 * 512], np.float32)},
                    "stereo_params": C.fisheye_stereo_params(), "map": mp,
                    "search": [{"cam": scam(camL, Rs, ts), "image": "left", "grid": (64, 48),
                                "preassigned": pre, "use_u_right": False},
                               {"cam": scam(camR, Rr, tr), "image": "right", "grid": (64, 48),
                                "preassigned": (r.random(n_kp) < 0.1).astype(np.uint8),
                                "use_u_right": False}],
                    "search_params": C.search_params(2.0),
                }
            frames.append(frame)
        st = {"id": s, "kind": str(kinds[s]), "rate_hz": rate, "n_map": n_map,
              "n_kp": n_kp, "frames": frames, "map_bytes": 64 * n_map}
        if edits is not None:
            st.update(points=table, map_ids0=id_sets[0], edits=edits)
        streams.append(st)
    return streams


def poisson_arrivals(rng, streams, duration_s: float, speedup: float = 1.0):
    """Sorted (time, stream, seq) arrivals: exponential gaps with mean
    1/(rate * speedup) per stream."""
    ev = []
    for s in streams:
        lam = s["rate_hz"] * speedup
        t = rng.exponential(1.0 / lam)
        k = 0
        while t < duration_s:
            ev.append((t, s["id"], k))
            k += 1
            t += rng.exponential(1.0 / lam)
    ev.sort()
    return ev
