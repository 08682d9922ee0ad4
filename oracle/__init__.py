"""CPU oracle of the tracking correspondence search (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never links or calls it, and it shares no
code with the device path: the C source (ft_oracle.c) is plain, single
threaded, and evaluates every definition as an exhaustive scan.

Functions take the frame dictionaries of the `synth` generators and return
numpy arrays.  Each one follows the paper's statement of the problem:
  stereo_pinhole       Section II-B (epipolar restriction) + IV-C (refine
                       among nearby pixels)
  stereo_fisheye       Section II-B (brute force) + IV-C (single kernel)
  search_local_points  Section II-D (Search by Projection) + IV-E
The numeric readings where the paper is silent are listed in ft_oracle.h's
header and in the project design notes.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, os.path.join(_HERE, "ft_oracle.c"), "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            src = os.path.join(_HERE, "ft_oracle.c")
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
                build()
            _lib = ct.CDLL(_SO)
            _lib.oracle_hamming.restype = ct.c_int
            _lib.oracle_kb_unproject.restype = ct.c_int
            _lib.oracle_triangulate.restype = ct.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _kp(kp):
    return (len(kp["x"]), _c(kp["x"], np.float32), _c(kp["y"], np.float32),
            _c(kp["octave"], np.uint8), _c(kp["desc"], np.uint8))


def hamming(a, b) -> int:
    a = _c(a, np.uint8); b = _c(b, np.uint8)
    return int(_load().oracle_hamming(_p(a), _p(b)))


def kb_array(cam) -> np.ndarray:
    return np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"], *list(cam["k"])], np.float32)


def kb_project(cam, X) -> np.ndarray:
    kb = kb_array(cam)
    X = _c(X, np.float64)
    uv = np.zeros(2, np.float64)
    _load().oracle_kb_project(_p(kb), _p(X), _p(uv))
    return uv


def kb_unproject(cam, u, v, iters=10, tol=1e-12, max_theta=np.deg2rad(88.0)):
    kb = kb_array(cam)
    ray = np.zeros(3, np.float64)
    ok = _load().oracle_kb_unproject(_p(kb), ct.c_float(u), ct.c_float(v), ct.c_int(iters),
                                     ct.c_double(tol), ct.c_double(max_theta), _p(ray))
    return (ray if ok else None)


def triangulate(r1, r2, R_lr, t_lr):
    r1 = _c(r1, np.float64); r2 = _c(r2, np.float64)
    R = _c(R_lr, np.float32).reshape(-1); t = _c(t_lr, np.float32)
    X = np.zeros(3, np.float64)
    ok = _load().oracle_triangulate(_p(r1), _p(r2), _p(R), _p(t), _p(X))
    return X if ok else None


def _cam_array(c) -> np.ndarray:
    return np.array([c["fx"], c["fy"], c["cx"], c["cy"], *list(c["k"]), c["bf"]], np.float32)


def search_last_frame(case) -> dict:
    """Search by projection of the last frame's matched map points into the
    current frame (Section II-C, Initial Pose Estimation), for a case from
    synth.last_frame_case."""
    lib = _load()
    last, kps, c, prm = case["last"], case["kps"], case["cam"], case["params"]
    nL = len(last["octave"])
    nK, kx, ky, ko, kd = _kp(kps)
    lpos = _c(last["pos"], np.float32); ld = _c(last["desc"], np.uint8)
    lo = _c(last["octave"], np.uint8); la = _c(last["angle"], np.float32)
    ka = _c(kps["angle"], np.float32)
    ur = None if case.get("u_right") is None else _c(case["u_right"], np.float32)
    pre = None if case.get("preassigned") is None else _c(case["preassigned"], np.uint8)
    cam = _cam_array(c)
    R = _c(c["R"], np.float32).reshape(-1); t = _c(c["t"], np.float32)
    bounds = _c(c["bounds"], np.float32)
    sf = _c(case["scales"]["sf"], np.float32)
    fp = np.array([prm["th"]], np.float32)
    ip = np.array([prm["th_high"], prm["direction"], prm["check_orientation"], prm["bins"]], np.int32)
    out = {"last_match": np.empty(nL, np.int32), "last_dist": np.empty(nL, np.int32),
           "kp_match": np.empty(nK, np.int32)}
    stats = np.zeros(8, np.int64)
    lib.oracle_search_last_frame(
        ct.c_int(nL), _p(lpos), _p(ld), _p(lo), _p(la),
        ct.c_int(nK), _p(kx), _p(ky), _p(ko), _p(kd), _p(ka), _p(ur), _p(pre),
        ct.c_int(int(c["model"])), _p(cam), _p(R), _p(t), _p(bounds), _p(sf), ct.c_int(len(sf)),
        _p(fp), _p(ip), _p(out["last_match"]), _p(out["last_dist"]), _p(out["kp_match"]), _p(stats))
    out["stats"] = dict(zip(["in_image", "candidates", "accepted", "after_conflict", "matches"],
                            stats[:5].tolist()))
    out["kept_bins"] = [int(b) for b in stats[5:8] if b >= 0]
    out["n_matches"] = int(stats[4])
    return out


def rotation_bin(a_last: float, a_cur: float, bins: int = 30) -> int:
    lib = _load()
    lib.oracle_rotation_bin.restype = ct.c_int
    return int(lib.oracle_rotation_bin(ct.c_float(a_last), ct.c_float(a_cur), ct.c_int(bins)))


def three_fullest(count) -> np.ndarray:
    cnt = _c(count, np.int32)
    kept = np.zeros(len(cnt), np.int32)
    _load().oracle_three_fullest(_p(cnt), ct.c_int(len(cnt)), _p(kept))
    return kept.astype(bool)


def map_update(mp: dict, capacity: int, remove, insert: dict | None):
    """Local-map maintenance in place (see ft_oracle.h): returns the edited
    map (arrays of length new n) or None when the edit is rejected."""
    n = len(mp["dmin"])
    m = 0 if insert is None else len(insert["dmin"])
    cap = max(capacity, 1)
    work = {"pos": np.zeros((cap, 3), np.float32), "normal": np.zeros((cap, 3), np.float32),
            "dmin": np.zeros(cap, np.float32), "dmax": np.zeros(cap, np.float32),
            "desc": np.zeros((cap, 32), np.uint8)}
    for k in work:
        work[k][:n] = mp[k]
    ins = insert if insert is not None else {k: v[:0] for k, v in work.items()}
    ins = {k: _c(v, work[k].dtype) for k, v in ins.items()}
    rem = _c(np.asarray(remove, np.int64), np.int32)
    lib = _load()
    new_n = lib.oracle_map_update(ct.c_int(n), ct.c_int(capacity), _p(work["pos"]), _p(work["normal"]),
                                  _p(work["dmin"]), _p(work["dmax"]), _p(work["desc"]), ct.c_int(len(rem)), _p(rem),
                                  ct.c_int(m), _p(ins["pos"]), _p(ins["normal"]), _p(ins["dmin"]), _p(ins["dmax"]),
                                  _p(ins["desc"]))
    if new_n < 0:
        return None
    return {k: np.ascontiguousarray(v[:new_n]) for k, v in work.items()}


def pyramid_layout(W: int, H: int, inv_sf) -> dict:
    """Level sizes and packed offsets of the image pyramid (Section IV-B)."""
    isf = _c(inv_sf, np.float32)
    n = len(isf)
    w = np.zeros(n, np.int32); h = np.zeros(n, np.int32); off = np.zeros(n, np.int64)
    lib = _load()
    lib.oracle_pyramid_layout.restype = ct.c_int64
    total = lib.oracle_pyramid_layout(ct.c_int(W), ct.c_int(H), _p(isf), ct.c_int(n), _p(w), _p(h), _p(off))
    return {"width": w, "height": h, "offset": off, "bytes": int(total)}


def pyramid(img, inv_sf) -> dict:
    """The image pyramid of a level-0 image (u8, H x W): every level computed
    from level 0, packed row-major level after level."""
    img = _c(img, np.uint8)
    H, W = img.shape
    lay = pyramid_layout(W, H, inv_sf)
    isf = _c(inv_sf, np.float32)
    out = np.zeros(lay["bytes"], np.uint8)
    _load().oracle_pyramid(_p(img), ct.c_int(W), ct.c_int(H), ct.c_int(W), _p(isf), ct.c_int(len(isf)),
                           _p(out))
    return {"data": out, "offset": lay["offset"], "width": lay["width"], "height": lay["height"]}


def fast_score_map(img, t: int, edge: int) -> np.ndarray:
    """FAST-9 scores of one image (u8, H x W): the score inside the detection
    window where it reaches t, 0 elsewhere (ORB extraction, Section II-A)."""
    img = _c(img, np.uint8)
    H, W = img.shape
    out = np.zeros((H, W), np.uint8)
    _load().oracle_fast_score_map(_p(img), ct.c_int(W), ct.c_int(H), ct.c_int(t), ct.c_int(edge), _p(out))
    return out


def orb_detect(pyr: dict, sf, t: int = 20, edge: int = 19, cap: int | None = None) -> dict:
    """Corners of every pyramid level after non-maximum suppression, in
    (level, y, x) order; `count` is the number found (at most `cap` written)."""
    lib = _load()
    lib.oracle_orb_detect.restype = ct.c_int64
    off = _c(pyr["offset"], np.int64); w = _c(pyr["width"], np.int32); h = _c(pyr["height"], np.int32)
    data = _c(pyr["data"], np.uint8)
    sff = _c(sf, np.float32)
    if cap is None:
        cap = int(np.sum(np.maximum(w.astype(np.int64) - 2 * edge, 0) * np.maximum(h.astype(np.int64) - 2 * edge, 0)))
    cap = max(int(cap), 0)
    out = {"lx": np.zeros(cap, np.int16), "ly": np.zeros(cap, np.int16), "octave": np.zeros(cap, np.uint8),
           "score": np.zeros(cap, np.uint8), "x": np.zeros(cap, np.float32), "y": np.zeros(cap, np.float32)}
    n = lib.oracle_orb_detect(_p(data), _p(off), _p(w), _p(h), ct.c_int(len(w)), _p(sff), ct.c_int(t),
                              ct.c_int(edge), ct.c_int64(cap), _p(out["lx"]), _p(out["ly"]), _p(out["octave"]),
                              _p(out["score"]), _p(out["x"]), _p(out["y"]))
    k = min(int(n), cap)
    res = {key: v[:k].copy() for key, v in out.items()}
    res["count"] = int(n)
    return res


def orb_blur(img) -> np.ndarray:
    """The descriptor's smoothing of one image (u8, H x W)."""
    img = _c(img, np.uint8)
    H, W = img.shape
    out = np.zeros((H, W), np.uint8)
    _load().oracle_orb_blur(_p(img), ct.c_int(W), ct.c_int(H), _p(out))
    return out


def orb_blur_pyramid(pyr: dict) -> np.ndarray:
    """Every level of a pyramid smoothed, in the pyramid's packed layout."""
    out = np.zeros_like(_c(pyr["data"], np.uint8))
    for l in range(len(pyr["width"])):
        w, h, o = int(pyr["width"][l]), int(pyr["height"][l]), int(pyr["offset"][l])
        out[o:o + w * h] = orb_blur(pyr["data"][o:o + w * h].reshape(h, w)).reshape(-1)
    return out


def orb_describe(pyr: dict, blurred, kps: dict, pattern) -> dict:
    """Orientation (degrees) and 256-bit descriptor of each keypoint (lx, ly,
    octave on the pyramid levels) with the point-pair `pattern` (int8 [256, 4])."""
    n = len(kps["lx"])
    off = _c(pyr["offset"], np.int64); w = _c(pyr["width"], np.int32)
    out = {"angle": np.zeros(n, np.float32), "desc": np.zeros((n, 32), np.uint8)}
    _load().oracle_orb_describe(_p(_c(pyr["data"], np.uint8)), _p(_c(blurred, np.uint8)), _p(off), _p(w),
                                ct.c_int(n), _p(_c(kps["lx"], np.int16)), _p(_c(kps["ly"], np.int16)),
                                _p(_c(kps["octave"], np.uint8)), _p(_c(pattern, np.int8)), _p(out["angle"]),
                                _p(out["desc"]))
    return out


def stereo_pinhole(frame) -> dict:
    lib = _load()
    nL, xL, yL, oL, dL = _kp(frame["left"])
    nR, xR, yR, oR, dR = _kp(frame["right"])
    pl, pr = frame["pyr_left"], frame["pyr_right"]
    sc = frame["scales"]
    cam = frame["stereo_cam"]
    sp = frame["stereo_params"]
    ip = np.array([sp["th_orb"], sp["half_win"], sp["half_range"], sp["level_window"],
                   sp["median_num"], sp["median_den"]], np.int32)
    out = {"right_idx": np.empty(nL, np.int32), "dist": np.empty(nL, np.int32),
           "u_right": np.empty(nL, np.float32), "depth": np.empty(nL, np.float32),
           "sad": np.empty(nL, np.int32)}
    stats = np.zeros(8, np.int64)
    pdl, pdr = _c(pl["data"], np.uint8), _c(pr["data"], np.uint8)
    off = _c(pl["offset"], np.int64); w = _c(pl["width"], np.int32); h = _c(pl["height"], np.int32)
    sf = _c(sc["sf"], np.float32); isf = _c(sc["inv_sf"], np.float32)
    lib.oracle_stereo_pinhole(
        ct.c_int(nL), _p(xL), _p(yL), _p(oL), _p(dL),
        ct.c_int(nR), _p(xR), _p(yR), _p(oR), _p(dR),
        _p(pdl), _p(pdr), _p(off), _p(w), _p(h), _p(sf), _p(isf),
        ct.c_float(cam["bf"]), ct.c_float(cam["b"]), ct.c_int(int(cam["rows"])), _p(ip),
        ct.c_float(sp["band"]),
        _p(out["right_idx"]), _p(out["dist"]), _p(out["u_right"]), _p(out["depth"]),
        _p(out["sad"]), _p(stats))
    out["stats"] = dict(zip(["hamming", "refine_attempts", "refined_ok", "after_conflict",
                             "median", "matches"], stats[:6].tolist()))
    out["n_matches"] = int(stats[5])
    return out


def stereo_fisheye(frame) -> dict:
    lib = _load()
    nL, xL, yL, oL, dL = _kp(frame["left"])
    nR, xR, yR, oR, dR = _kp(frame["right"])
    cam = frame["stereo_cam"]
    sp = frame["stereo_params"]
    kbl, kbr = kb_array(cam["left"]), kb_array(cam["right"])
    R = _c(cam["R_lr"], np.float32).reshape(-1); t = _c(cam["t_lr"], np.float32)
    ovl = _c(cam["overlap_left"], np.float32); ovr = _c(cam["overlap_right"], np.float32)
    s2 = _c(frame["scales"]["sigma2"], np.float32)
    ip = np.array([sp["ratio_num"], sp["ratio_den"], sp["newton_iters"]], np.int32)
    dp = np.array([sp["cos_parallax_max"], sp["chi2"], np.deg2rad(sp["max_theta_deg"]),
                   sp["newton_tol"]], np.float64)
    out = {"right_idx": np.empty(nL, np.int32), "dist": np.empty(nL, np.int32),
           "depth": np.empty(nL, np.float32), "xyz": np.empty((nL, 3), np.float32),
           "h2": np.empty(nL, np.int32)}
    stats = np.zeros(8, np.int64)
    lib.oracle_stereo_fisheye(
        ct.c_int(nL), _p(xL), _p(yL), _p(oL), _p(dL),
        ct.c_int(nR), _p(xR), _p(yR), _p(oR), _p(dR),
        _p(kbl), _p(kbr), _p(R), _p(t), _p(ovl), _p(ovr), _p(s2), _p(ip), _p(dp),
        _p(out["right_idx"]), _p(out["dist"]), _p(out["depth"]), _p(out["xyz"]), _p(out["h2"]), _p(stats))
    out["stats"] = dict(zip(["Q", "T", "ratio_ok", "tri_ok", "matches", "rej_parallax", "rej_depth",
                             "rej_reproj"], stats.tolist()))
    out["n_matches"] = int(stats[4])
    return out


def search_params_arrays(sp):
    fp = np.array([sp["th"], sp["view_cos_limit"], sp["view_cos_narrow"], sp["r_narrow"],
                   sp["r_wide"], sp["dist_lo"], sp["dist_hi"]], np.float32)
    ip = np.array([sp["level_lo"], sp["level_hi"], sp["th_high"], sp["ratio_num"],
                   sp["ratio_den"], sp["ratio_same_level_only"]], np.int32)
    return fp, ip


def search_local_points(frame, view: int = 0, u_right=None) -> dict:
    """Search by projection for one camera view of `frame` (view 0 = left)."""
    lib = _load()
    spec = frame["search"][view]
    kp = frame[spec["image"]]
    nK, kx, ky, ko, kd = _kp(kp)
    mp = frame["map"]
    nM = len(mp["dmin"])
    pos = _c(mp["pos"], np.float32); nrm = _c(mp["normal"], np.float32)
    dmin = _c(mp["dmin"], np.float32); dmax = _c(mp["dmax"], np.float32)
    mdesc = _c(mp["desc"], np.uint8)
    cam = spec["cam"]
    camv = np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"], *list(cam["k"]), cam["bf"]],
                    np.float32)
    R = _c(cam["R"], np.float32).reshape(-1); t = _c(cam["t"], np.float32)
    O = _c(cam["O"], np.float32); bounds = _c(cam["bounds"], np.float32)
    sf = _c(frame["scales"]["sf"], np.float32)
    fp, ip = search_params_arrays(frame["search_params"])
    ur = None if u_right is None else _c(u_right, np.float32)
    pre = None if spec.get("preassigned") is None else _c(spec["preassigned"], np.uint8)
    out = {"mp_match": np.empty(nM, np.int32), "mp_dist": np.empty(nM, np.int32),
           "kp_match": np.empty(nK, np.int32)}
    stats = np.zeros(8, np.int64)
    lib.oracle_search_local_points(
        ct.c_int(nM), _p(pos), _p(nrm), _p(dmin), _p(dmax), _p(mdesc),
        ct.c_int(nK), _p(kx), _p(ky), _p(ko), _p(kd), _p(ur), _p(pre),
        ct.c_int(int(cam["model"])), _p(camv), _p(R), _p(t), _p(O), _p(bounds), _p(sf),
        ct.c_int(len(sf)), _p(fp), _p(ip),
        _p(out["mp_match"]), _p(out["mp_dist"]), _p(out["kp_match"]), _p(stats))
    out["stats"] = dict(zip(["visible", "candidates", "accepted", "matches", "rej_frame", "rej_near",
                             "rej_far", "rej_angle"], stats.tolist()))
    out["n_matches"] = int(stats[3])
    return out


def run_frame(frame) -> dict:
    """The whole per-frame hot path: stereo matching, then search by projection
    in every camera view (the pinhole view gates candidates with the stereo
    right coordinates)."""
    res = {"kind": frame["kind"]}
    if frame["kind"] == "pinhole":
        st = stereo_pinhole(frame)
        res["stereo"] = st
        res["search"] = [search_local_points(frame, 0, st["u_right"])]
    elif frame["kind"] == "fisheye":
        res["stereo"] = stereo_fisheye(frame)
        res["search"] = [search_local_points(frame, v) for v in range(len(frame["search"]))]
    else:
        res["search"] = [search_local_points(frame, v) for v in range(len(frame["search"]))]
    return res


def sad_window(IL, IR, su, sv, su0, w=5, L=5):
    """Centre-subtracted SAD profile for shifts -L..L, or None when out of bounds."""
    IL = _c(IL, np.uint8); IR = _c(IR, np.uint8)
    H, W = IL.shape
    sad = np.zeros(2 * L + 1, np.int32)
    ok = _load().oracle_sad_window(_p(IL), _p(IR), ct.c_int(W), ct.c_int(H), ct.c_int(su),
                                   ct.c_int(sv), ct.c_int(su0), ct.c_int(w), ct.c_int(L), _p(sad))
    return sad if ok else None


def subpixel(sad, L=5):
    """(best shift, its SAD, parabola vertex offset) or None when rejected."""
    sad = _c(sad, np.int32)
    kb = ct.c_int(); c = ct.c_int(); d = ct.c_float()
    ok = _load().oracle_subpixel(_p(sad), ct.c_int(L), ct.byref(kb), ct.byref(c), ct.byref(d))
    return (kb.value, c.value, d.value) if ok else None


def median_keep(sad, num=21, den=10):
    sad = _c(sad, np.int32)
    keep = np.zeros(max(len(sad), 1), np.uint8)
    m = _load().oracle_median_keep(ct.c_int(len(sad)), _p(sad), ct.c_int(num), ct.c_int(den),
                                   _p(keep))
    return int(m), keep[:len(sad)].astype(bool)


def predict_level(ratio, sf):
    sf = _c(sf, np.float32)
    return int(_load().oracle_predict_level(ct.c_float(ratio), _p(sf), ct.c_int(len(sf))))


class using_library:
    """Temporarily route every oracle call to another build of ft_oracle.c
    (used by the tests that plant mistakes in a copy of the oracle)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self._saved = _lib
        lib = ct.CDLL(self.path)
        lib.oracle_hamming.restype = ct.c_int
        lib.oracle_kb_unproject.restype = ct.c_int
        lib.oracle_triangulate.restype = ct.c_int
        _lib = lib
        return lib

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False
