"""Vectorised numpy brute force of the matching definitions, for tiny inputs.

Independent of the C oracle (no shared code): every candidate predicate is
evaluated for ALL (query, target) pairs as a boolean matrix, distances come
from numpy.unpackbits, best/second come from sorting (distance, index) keys,
and patches are cut with array slicing.  Binary32 arithmetic is reproduced by
numpy float32 ufuncs (separate multiply and add, so no fused multiply-add).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def bits(desc):
    return np.unpackbits(np.asarray(desc, np.uint8), axis=1, bitorder="little").astype(np.int32)


def hamming_matrix(a, b):
    A, B = bits(a), bits(b)
    return (A[:, None, :] != B[None, :, :]).sum(-1).astype(np.int64)


def round_half_away(x):
    x = np.asarray(x, np.float64)
    return np.where(x >= 0, np.floor(x + 0.5), -np.floor(-x + 0.5)).astype(np.int64)


def lexmin2(valid, H):
    """Per row: (H1, k1, H2, k2) lexicographic minima of (H, k) over valid cells."""
    n, m = H.shape
    big = np.int64(1) << 40
    key = np.where(valid, H * (m + 1) + np.arange(m)[None, :], big)
    order = np.argsort(key, axis=1, kind="stable")
    k1 = order[:, 0] if m else np.zeros(n, np.int64)
    k2 = order[:, 1] if m > 1 else np.full(n, -1)
    has1 = valid.any(1)
    has2 = valid.sum(1) >= 2
    H1 = np.where(has1, H[np.arange(n), k1] if m else 0, -1)
    H2 = np.where(has2, H[np.arange(n), np.maximum(k2, 0)] if m > 1 else 0, -1)
    return np.where(has1, H1, -1), np.where(has1, k1, -1), H2, np.where(has2, k2, -1)


def resolve(target, dist, alive, n_targets):
    """Keep, for every target, only the claim with the smallest (dist, query)."""
    alive = alive.copy()
    q = np.nonzero(alive)[0]
    if q.size == 0:
        return alive
    key = dist[q].astype(np.int64) * (1 << 32) + q
    best = np.full(n_targets, np.iinfo(np.int64).max)
    np.minimum.at(best, target[q], key)
    alive[q] = best[target[q]] == key
    return alive


def level_image(pyr, l):
    o = int(pyr["offset"][l]); w = int(pyr["width"][l]); h = int(pyr["height"][l])
    return pyr["data"][o:o + w * h].reshape(h, w).astype(np.int64)


def sad_profile(IL, IR, su, sv, su0, w, L):
    H, W = IL.shape
    if su - w < 0 or su + w >= W or sv - w < 0 or sv + w >= H or su0 - L - w < 0 or su0 + L + w >= W:
        return None
    pl = IL[sv - w:sv + w + 1, su - w:su + w + 1] - IL[sv, su]
    out = []
    for k in range(-L, L + 1):
        pr = IR[sv - w:sv + w + 1, su0 + k - w:su0 + k + w + 1] - IR[sv, su0 + k]
        out.append(int(np.abs(pl - pr).sum()))
    return np.array(out, np.int64)


def stereo_pinhole(frame):
    Lk, Rk = frame["left"], frame["right"]
    sc, cam, sp = frame["scales"], frame["stereo_cam"], frame["stereo_params"]
    sf, isf = sc["sf"], sc["inv_sf"]
    xL, yL, oL = Lk["x"], Lk["y"], Lk["octave"].astype(np.int64)
    xR, yR, oR = Rk["x"], Rk["y"], Rk["octave"].astype(np.int64)
    nL, nR = len(xL), len(xR)
    rows = int(cam["rows"])
    maxD = f32(cam["bf"]) / f32(cam["b"])
    r = f32(sp["band"]) * sf[oR]
    lo = np.maximum(np.floor(yR - r).astype(np.int64), 0)
    hi = np.minimum(np.ceil(yR + r).astype(np.int64), rows - 1)
    row = np.trunc(yL).astype(np.int64)
    minU = xL - maxD
    maxU = xL - f32(0.0)
    lw = sp["level_window"]
    P = ((row[:, None] >= lo[None, :]) & (row[:, None] <= hi[None, :]) &
         (np.abs(oL[:, None] - oR[None, :]) <= lw) &
         (xR[None, :] >= minU[:, None]) & (xR[None, :] <= maxU[:, None]) &
         (maxU >= 0)[:, None])
    Hm = hamming_matrix(Lk["desc"], Rk["desc"])
    H1, j1, _, _ = lexmin2(P, Hm)
    cand = (j1 >= 0) & (H1 < sp["th_orb"])

    w, Lr = sp["half_win"], sp["half_range"]
    res_j = np.full(nL, -1); res_h = np.full(nL, -1); res_s = np.full(nL, -1)
    res_u = np.full(nL, -1, np.float32); res_d = np.full(nL, -1, np.float32)
    alive = np.zeros(nL, bool)
    n_hamming = int(P.sum())
    for i in np.nonzero(cand)[0]:
        l = int(oL[i]); s = isf[l]
        su = int(round_half_away(xL[i] * s)); sv = int(round_half_away(yL[i] * s))
        su0 = int(round_half_away(xR[j1[i]] * s))
        prof = sad_profile(level_image(frame["pyr_left"], l), level_image(frame["pyr_right"], l),
                           su, sv, su0, w, Lr)
        if prof is None:
            continue
        kb = int(np.argmin(prof)) - Lr
        if abs(kb) == Lr:
            continue
        a, c, e = prof[kb + Lr - 1], prof[kb + Lr], prof[kb + Lr + 1]
        delta = f32(a - e) / f32(2 * (a + e - 2 * c))
        if delta < -1 or delta > 1:
            continue
        uR = sf[l] * ((f32(su0) + f32(kb)) + delta)
        disp = xL[i] - uR
        if not (disp >= f32(0) and disp < maxD):
            continue
        if disp <= 0:
            disp = f32(0.01)
            uR = f32(np.float64(xL[i]) - 0.01)
        res_j[i], res_h[i], res_s[i] = j1[i], H1[i], c
        res_u[i], res_d[i] = uR, f32(cam["bf"]) / disp
        alive[i] = True
    alive = resolve(res_j, res_h, alive, nR)
    q = np.nonzero(alive)[0]
    keep = np.zeros(nL, bool)
    median = -1
    if q.size:
        median = int(np.sort(res_s[q])[q.size // 2])
        keep[q] = sp["median_den"] * res_s[q] < sp["median_num"] * median
    out = {"right_idx": np.where(keep, res_j, -1), "dist": np.where(keep, res_h, -1),
           "u_right": np.where(keep, res_u, f32(-1)), "depth": np.where(keep, res_d, f32(-1)),
           "sad": np.where(keep, res_s, -1)}
    out["stats"] = {"hamming": n_hamming, "after_conflict": int(q.size), "median": median}
    return out


def knn2_overlap(frame):
    """Fisheye kNN stage: top-2 over the right overlap for left overlap queries,
    and the ratio decision."""
    Lk, Rk, cam, sp = frame["left"], frame["right"], frame["stereo_cam"], frame["stereo_params"]
    a_l, b_l = cam["overlap_left"]; a_r, b_r = cam["overlap_right"]
    Q = (Lk["x"] >= a_l) & (Lk["x"] <= b_l)
    T = (Rk["x"] >= a_r) & (Rk["x"] <= b_r)
    Hm = hamming_matrix(Lk["desc"], Rk["desc"])
    valid = Q[:, None] & T[None, :]
    H1, j1, H2, _ = lexmin2(valid, Hm)
    ratio_ok = Q & (T.sum() >= 2) & (sp["ratio_den"] * H1 < sp["ratio_num"] * H2)
    return H1, j1, H2, ratio_ok


def search_pinhole(frame, view=0, u_right=None):
    """Search by projection, pinhole model, every (map point, keypoint) pair."""
    spec = frame["search"][view]
    kp = frame[spec["image"]]
    mp = frame["map"]
    cam = spec["cam"]
    sp = frame["search_params"]
    sf = frame["scales"]["sf"]
    R, t, O = cam["R"], cam["t"], cam["O"]
    X, Y, Z = mp["pos"][:, 0], mp["pos"][:, 1], mp["pos"][:, 2]
    xc = ((R[0, 0] * X + R[0, 1] * Y) + R[0, 2] * Z) + t[0]
    yc = ((R[1, 0] * X + R[1, 1] * Y) + R[1, 2] * Z) + t[1]
    zc = ((R[2, 0] * X + R[2, 1] * Y) + R[2, 2] * Z) + t[2]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = ((cam["fx"] * xc) / zc) + cam["cx"]
        v = ((cam["fy"] * yc) / zc) + cam["cy"]
        b = cam["bounds"]
        pox, poy, poz = X - O[0], Y - O[1], Z - O[2]
        dist = np.sqrt((pox * pox + poy * poy) + poz * poz)
        vcos = ((pox * mp["normal"][:, 0] + poy * mp["normal"][:, 1]) + poz * mp["normal"][:, 2]) / dist
        ratio = mp["dmax"] / dist
    in_frame = (zc > 0) & (u >= b[0]) & (u <= b[1]) & (v >= b[2]) & (v <= b[3])
    near_ok = dist >= f32(sp["dist_lo"]) * mp["dmin"]
    far_ok = dist <= f32(sp["dist_hi"]) * mp["dmax"]
    angle_ok = vcos >= f32(sp["view_cos_limit"])
    vis = in_frame & near_ok & far_ok & angle_ok
    reach = sf[None, :] >= ratio[:, None]
    pred = np.where(reach.any(1), np.argmax(reach, axis=1), len(sf) - 1)
    rbase = np.where(vcos > f32(sp["view_cos_narrow"]), f32(sp["r_narrow"]), f32(sp["r_wide"])) * f32(sp["th"])
    Rm = (rbase * sf[pred]).astype(np.float32)
    ko = kp["octave"].astype(np.int64)
    with np.errstate(invalid="ignore", over="ignore"):
        C = (vis[:, None] &
             (ko[None, :] >= pred[:, None] - sp["level_lo"]) & (ko[None, :] <= pred[:, None] + sp["level_hi"]) &
             (np.abs(kp["x"][None, :] - u[:, None]) < Rm[:, None]) &
             (np.abs(kp["y"][None, :] - v[:, None]) < Rm[:, None]))
        if spec.get("preassigned") is not None:
            C &= ~spec["preassigned"].astype(bool)[None, :]
        if u_right is not None:
            uR = u - cam["bf"] * (f32(1.0) / zc)
            gate = (u_right[None, :] > 0) & ~(np.abs(uR[:, None] - u_right[None, :]) <= Rm[:, None])
            C &= ~gate
    Hm = hamming_matrix(mp["desc"], kp["desc"])
    H1, k1, H2, k2 = lexmin2(C, Hm)
    l1 = np.where(k1 >= 0, ko[np.maximum(k1, 0)], -1)
    l2 = np.where(k2 >= 0, ko[np.maximum(k2, 0)], -1)
    H2 = np.where(k2 >= 0, H2, 256)
    fails = sp["ratio_den"] * H1 > sp["ratio_num"] * H2
    if sp["ratio_same_level_only"]:
        fails = fails & (l1 == l2)
    acc = (k1 >= 0) & (H1 <= sp["th_high"]) & ~fails
    alive = resolve(k1, H1, acc, len(kp["x"]))
    mp_match = np.where(alive, k1, -1)
    kp_match = np.full(len(kp["x"]), -1)
    kp_match[k1[alive]] = np.nonzero(alive)[0]
    return {"mp_match": mp_match, "mp_dist": np.where(alive, H1, -1), "kp_match": kp_match,
            "stats": {"visible": int(vis.sum()), "candidates": int(C.sum()),
                      "accepted": int(acc.sum()), "matches": int(alive.sum()),
                      "rej_frame": int((~in_frame).sum()), "rej_near": int((in_frame & ~near_ok).sum()),
                      "rej_far": int((in_frame & near_ok & ~far_ok).sum()),
                      "rej_angle": int((in_frame & near_ok & far_ok & ~angle_ok).sum())}}


def rotation_bins(a_last, a_cur, bins):
    """Rotation bin of every match, binary32 as in the definition."""
    rot = (np.asarray(a_last, np.float32) - np.asarray(a_cur, np.float32)).astype(np.float32)
    rot = np.where(rot < 0, (rot + f32(360.0)).astype(np.float32), rot)
    b = round_half_away((rot * (f32(bins) / f32(360.0))).astype(np.float32))
    return np.mod(b, bins)


def three_fullest(count):
    """Kept bins: the fullest and, while 10 * count >= the fullest, the second
    and third fullest; ties go to the lower bin (stable sort by -count)."""
    count = np.asarray(count, np.int64)
    order = np.argsort(-count, kind="stable")
    kept = np.zeros(len(count), bool)
    if len(count) == 0 or count[order[0]] == 0:
        return kept
    m1 = count[order[0]]
    kept[order[0]] = True
    for j in (1, 2):
        if j < len(count) and count[order[j]] > 0 and 10 * count[order[j]] >= m1:
            kept[order[j]] = True
        else:
            break
    return kept


def search_last_frame_pinhole(case):
    """Last-frame search by projection (pinhole camera) over every (point,
    keypoint) pair."""
    last, kp, cam, prm = case["last"], case["kps"], case["cam"], case["params"]
    sf = case["scales"]["sf"]
    nL, nK = len(last["octave"]), len(kp["x"])
    R, t = cam["R"], cam["t"]
    P = last["pos"]
    X, Y, Z = P[:, 0], P[:, 1], P[:, 2]
    xc = ((R[0, 0] * X + R[0, 1] * Y) + R[0, 2] * Z) + t[0]
    yc = ((R[1, 0] * X + R[1, 1] * Y) + R[1, 2] * Z) + t[1]
    zc = ((R[2, 0] * X + R[2, 1] * Y) + R[2, 2] * Z) + t[2]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = ((cam["fx"] * xc) / zc) + cam["cx"]
        v = ((cam["fy"] * yc) / zc) + cam["cy"]
    b = cam["bounds"]
    inside = (zc > 0) & (u >= b[0]) & (u <= b[1]) & (v >= b[2]) & (v <= b[3])
    lo = last["octave"].astype(np.int64)
    r = (f32(prm["th"]) * sf[np.minimum(lo, len(sf) - 1)]).astype(np.float32)
    d = prm["direction"]
    lv_min = np.where(d > 0, lo, np.where(d < 0, 0, lo - 1))
    lv_max = np.where(d > 0, len(sf) - 1, np.where(d < 0, lo, lo + 1))
    ko = kp["octave"].astype(np.int64)
    with np.errstate(invalid="ignore", over="ignore"):
        C = (inside[:, None] & (ko[None, :] >= lv_min[:, None]) & (ko[None, :] <= lv_max[:, None]) &
             (np.abs(kp["x"][None, :] - u[:, None]) < r[:, None]) &
             (np.abs(kp["y"][None, :] - v[:, None]) < r[:, None]))
        if case.get("preassigned") is not None:
            C &= ~case["preassigned"].astype(bool)[None, :]
        if case.get("u_right") is not None:
            ur = case["u_right"]
            uR = u - cam["bf"] * (f32(1.0) / zc)
            C &= ~((ur[None, :] > 0) & ~(np.abs(uR[:, None] - ur[None, :]) <= r[:, None]))
    Hm = hamming_matrix(last["desc"], kp["desc"])
    H1, k1, _, _ = lexmin2(C, Hm)
    acc = (k1 >= 0) & (H1 <= prm["th_high"])
    alive = resolve(k1, H1, acc, nK)
    kept_bins = []
    if prm["check_orientation"]:
        q = np.nonzero(alive)[0]
        bins = rotation_bins(last["angle"][q], kp["angle"][k1[q]], prm["bins"])
        kept = three_fullest(np.bincount(bins, minlength=prm["bins"]))
        alive[q] = kept[bins]
        kept_bins = [int(x) for x in np.nonzero(kept)[0]]
    lm = np.where(alive, k1, -1)
    kp_match = np.full(nK, -1)
    kp_match[k1[alive]] = np.nonzero(alive)[0]
    return {"last_match": lm, "last_dist": np.where(alive, H1, -1), "kp_match": kp_match,
            "kept_bins": kept_bins,
            "stats": {"in_image": int(inside.sum()), "candidates": int(C.sum()),
                      "accepted": int(acc.sum()), "matches": int(alive.sum())}}
