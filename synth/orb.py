"""Seeded inputs of ORB extraction: the descriptor's point-pair pattern.

The pattern is an input of the extraction (the caller supplies it), drawn
here the way BRIEF draws its tests: both points of a pair from an isotropic
Gaussian around the keypoint with standard deviation patch / 5 (patch = 31
pixels), rounded to whole pixels and redrawn until the point lies within
radius 13 and the two points of the pair differ.
"""
from __future__ import annotations

import numpy as np

from . import common as C


def orb_pattern(seed=None, n_tests: int = 256, radius: int = 13, patch: int = 31) -> np.ndarray:
    """int8 [n_tests, 4] rows (x1, y1, x2, y2)."""
    rng = np.random.default_rng(seed if seed is not None else np.random.SeedSequence(C.MASTER_SEED + 31))
    out = np.zeros((n_tests, 4), np.int8)
    sigma = patch / 5.0

    def point():
        while True:
            p = np.rint(rng.normal(0.0, sigma, 2)).astype(int)
            if p[0] * p[0] + p[1] * p[1] <= radius * radius:
                return p
    for t in range(n_tests):
        while True:
            a, b = point(), point()
            if (a != b).any():
                break
        out[t] = (a[0], a[1], b[0], b[1])
    return out
