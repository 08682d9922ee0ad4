"""Map points that reach the visibility tests of search by projection.

The scene generators build every map point from a camera that saw it, so each
point lies inside its own distance range and is seen nearly along its mean
viewing direction.  A tracker's local map also holds points that the current
frame sees from too close, too far or from the side.  `add_gate_cases` turns a
seeded fraction of a frame's map points into such points, for each test:

  near   seen nearer than dist_lo * dmin     (dmin raised past dist / dist_lo)
  far    seen farther than dist_hi * dmax    (dmax lowered below dist / dist_hi)
  angle  viewing cosine below the limit      (normal turned 62-150 degrees off the ray)

plus points exactly on each boundary in binary32 (the last value that passes
and the first that fails), so that the comparison direction of every test is
exercised.  Only the map point record is changed (dmin, dmax or normal); the
position, descriptor and keypoints stay as generated.  Distances and cosines are
taken from the pose of search view 0, in the binary32 operation order the
visibility tests use (they only choose inputs here).
"""
from __future__ import annotations

import numpy as np

from . import common as C

f32 = np.float32


def _dist32(P, O):
    d = (P.astype(np.float32) - O.astype(np.float32)[None, :]).astype(np.float32)
    return np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]).astype(np.float32), d


def _cos32(d, n, dist):
    return (((d[:, 0] * n[:, 0] + d[:, 1] * n[:, 1]) + d[:, 2] * n[:, 2]) / dist).astype(np.float32)


def _last_passing_min(dist, lo):
    """Largest binary32 dmin with fl32(lo * dmin) <= dist."""
    d = f32(dist / lo)
    while f32(f32(lo) * d) > dist:
        d = np.nextafter(d, f32(0))
    while f32(f32(lo) * np.nextafter(d, f32(np.inf))) <= dist:
        d = np.nextafter(d, f32(np.inf))
    return d


def _first_passing_max(dist, hi):
    """Smallest binary32 dmax with fl32(hi * dmax) >= dist."""
    d = f32(dist / hi)
    while f32(f32(hi) * d) < dist:
        d = np.nextafter(d, f32(np.inf))
    while f32(f32(hi) * np.nextafter(d, f32(0))) >= dist:
        d = np.nextafter(d, f32(0))
    return d


def _turned_normal(ray, axis_seed, angle):
    """Unit vector at `angle` (radians) from the unit `ray`, about an axis
    perpendicular to it."""
    a = axis_seed - np.dot(axis_seed, ray) * ray
    a /= np.linalg.norm(a)
    return C.rodrigues(a, angle) @ ray


def _normal_on_cos_boundary(rng, d, dist, limit, inside):
    """A binary32 unit normal whose binary32 viewing cosine is the smallest value
    >= limit (inside) or the largest value < limit (outside)."""
    ray = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64))
    axis = C.random_unit(rng)
    base = np.arccos(float(limit))
    best = None
    for step in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        for k in range(-200, 201):
            ang = base + k * step if best is None else best[0] + k * step
            n = _turned_normal(ray, axis, ang).astype(np.float32)
            c = _cos32(d[None, :], n[None, :], np.array([dist], np.float32))[0]
            ok = (c >= limit) if inside else (c < limit)
            if not ok:
                continue
            gap = abs(float(c) - float(limit))
            if best is None or gap < best[1]:
                best = (ang, gap, n, c)
    return best[2], best[3]


def add_gate_cases(frame, seed, frac: float = 0.03, n_edge: int = 4):
    """Returns (frame, cases): a copy of `frame` whose map has `frac` of its
    points past each visibility test and `n_edge` points on each side of each
    test's boundary; `cases` maps a case name to the map point indices."""
    rng = np.random.default_rng(seed)
    out = dict(frame)
    mp = {k: v.copy() for k, v in frame["map"].items()}
    out["map"] = mp
    sp = frame["search_params"]
    lo, hi, cos_lim = f32(sp["dist_lo"]), f32(sp["dist_hi"]), f32(sp["view_cos_limit"])
    O = frame["search"][0]["cam"]["O"]
    dist, d = _dist32(mp["pos"], O)
    nM = len(dist)
    k = int(round(frac * nM))
    names = ["near", "far", "angle"]
    edges = ["near_in", "near_out", "far_in", "far_out", "angle_in", "angle_out"]
    sizes = [k] * len(names) + [n_edge] * len(edges)
    if sum(sizes) > nM:
        raise ValueError("map too small for the requested gate cases")
    perm = rng.permutation(nM)
    cases, at = {}, 0
    for name, n in zip(names + edges, sizes):
        cases[name] = np.sort(perm[at:at + n])
        at += n
    sf7 = float(frame["scales"]["sf"][-1])

    i = cases["near"]
    mp["dmin"][i] = (dist[i].astype(np.float64) / float(lo) * rng.uniform(1.02, 1.5, len(i))).astype(np.float32)
    i = cases["far"]
    mp["dmax"][i] = (dist[i].astype(np.float64) / float(hi) * rng.uniform(0.6, 0.98, len(i))).astype(np.float32)
    mp["dmin"][i] = (mp["dmax"][i].astype(np.float64) / sf7).astype(np.float32)
    i = cases["angle"]
    for m in i:
        ray = d[m].astype(np.float64) / np.linalg.norm(d[m].astype(np.float64))
        mp["normal"][m] = _turned_normal(ray, C.random_unit(rng), np.deg2rad(rng.uniform(62.0, 150.0)))

    for m in cases["near_in"]:
        mp["dmin"][m] = _last_passing_min(dist[m], lo)
    for m in cases["near_out"]:
        mp["dmin"][m] = np.nextafter(_last_passing_min(dist[m], lo), f32(np.inf))
    for m in cases["far_in"]:
        mp["dmax"][m] = _first_passing_max(dist[m], hi)
        mp["dmin"][m] = min(mp["dmin"][m], f32(float(mp["dmax"][m]) / sf7))
    for m in cases["far_out"]:
        mp["dmax"][m] = np.nextafter(_first_passing_max(dist[m], hi), f32(0))
        mp["dmin"][m] = min(mp["dmin"][m], f32(float(mp["dmax"][m]) / sf7))
    for name, inside in (("angle_in", True), ("angle_out", False)):
        for m in cases[name]:
            mp["normal"][m], _ = _normal_on_cos_boundary(rng, d[m], dist[m], cos_lim, inside)
    return out, cases


def gate_outcomes(frame, cases):
    """For the boundary cases: the binary32 test values as the generator set
    them (used by tests to check the cases really sit on the boundary)."""
    mp = frame["map"]
    sp = frame["search_params"]
    dist, d = _dist32(mp["pos"], frame["search"][0]["cam"]["O"])
    lo, hi = f32(sp["dist_lo"]), f32(sp["dist_hi"])
    res = {}
    for name in ("near_in", "near_out"):
        i = cases[name]
        res[name] = dist[i] >= (lo * mp["dmin"][i]).astype(np.float32)
    for name in ("far_in", "far_out"):
        i = cases[name]
        res[name] = dist[i] <= (hi * mp["dmax"][i]).astype(np.float32)
    for name in ("angle_in", "angle_out"):
        i = cases[name]
        res[name] = _cos32(d[i], mp["normal"][i], dist[i]) >= f32(sp["view_cos_limit"])
    return res
