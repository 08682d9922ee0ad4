"""Device local-map maintenance (ft_map_update) against the CPU oracle.

A map in device memory is edited in place by sequences of removals and
insertions (nothing, everything, head-only, tail-only, random mixes, exact
capacity) and must equal the oracle's edited map byte for byte after every
edit; a search by projection over an edited map equals the oracle's search over
the oracle's edited map; invalid edits are rejected with the map unchanged.
"""
import copy
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity import compare_search

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(ft):
    return ft.Context(ft.default_limits(max_batch_frames=1, max_map_points=32768, max_inflight=1))


def _points(n, seed, tag0):
    rng = np.random.default_rng(seed)
    return {"pos": rng.normal(0, 5, (n, 3)).astype(np.float32),
            "normal": rng.normal(0, 1, (n, 3)).astype(np.float32),
            "dmin": (tag0 + np.arange(n)).astype(np.float32),
            "dmax": rng.uniform(1, 20, n).astype(np.float32),
            "desc": rng.integers(0, 256, (n, 32), dtype=np.uint8)}


def _same(dev, want, tag):
    for k in want:
        assert np.array_equal(dev[k].view(np.uint8), want[k].view(np.uint8)), (tag, k)


def test_map_edit_sequences_equal_oracle(ft, ctx):
    rng = np.random.default_rng(11)
    cap = 6000
    mp = _points(4000, 12, 0)
    dm = ft.DeviceMap(mp, cap)
    tag = 100000
    # nothing; insert only; head only; tail only (no holes)
    edits = [lambda n: ([], 0), lambda n: ([], 50), lambda n: (list(range(10)), 0),
             lambda n: (list(range(n - 60, n)), 5)]
    for step in range(40):
        n = dm.n
        if step < len(edits):
            remove, m = edits[step](n)
        else:
            remove = rng.choice(n, int(rng.integers(0, min(n, 400) + 1)), replace=False).tolist()
            m = int(rng.integers(0, 400))
        if n - len(remove) + m > cap:
            m = cap - (n - len(remove))
        ins = _points(m, 200 + step, tag)
        tag += m
        say("edit", step, "n", n, "remove", len(remove), "insert", m)
        want = oracle.map_update(mp, cap, remove, ins)
        dm.edit(ctx, remove, ins)
        torch.cuda.synchronize()
        assert dm.n == len(want["dmin"])
        _same(dm.host(), want, step)
        mp = want
    # everything out, then refill to exact capacity
    want = oracle.map_update(mp, cap, list(range(dm.n)), _points(cap, 999, tag))
    dm.edit(ctx, list(range(dm.n)), _points(cap, 999, tag))
    torch.cuda.synchronize()
    assert dm.n == cap
    _same(dm.host(), want, "refill")


def test_invalid_edits_leave_the_map(ft, ctx):
    mp = _points(100, 21, 0)
    dm = ft.DeviceMap(mp, 120)
    for remove, m, status in (([3, 3], 0, ft.FT_ERR_INVALID_ARGUMENT), ([100], 0, ft.FT_ERR_INVALID_ARGUMENT),
                              ([-2], 0, ft.FT_ERR_INVALID_ARGUMENT), ([], 21, ft.FT_ERR_CAPACITY),
                              ([0], 22, ft.FT_ERR_CAPACITY)):
        assert dm.edit(ctx, remove, _points(m, 22, 500), check=False) == status, (remove, m)
        assert dm.n == 100
    torch.cuda.synchronize()
    _same(dm.host(), mp, "unchanged")


@pytest.mark.parametrize("kind", ["pinhole", "fisheye"])
def test_search_over_an_edited_map(ft, ctx, kind):
    """A frame's local map edited on the device (10% of its points removed,
    points of another frame's map inserted): the search over it equals the
    oracle's search over the oracle's edited map."""
    f = synth.pinhole_frame_1200()[0] if kind == "pinhole" else synth.fisheye_frame_1500()[0]
    other = synth.tiny_clustered(31, n_map=700)["map"] if kind == "pinhole" else synth.tiny_fisheye(31, n_map=600)["map"]
    n = len(f["map"]["dmin"])
    rng = np.random.default_rng(32)
    remove = rng.choice(n, n // 10, replace=False)
    cap = n + 1000
    want_map = oracle.map_update(f["map"], cap, remove, other)
    g = copy.copy(f)
    g["map"] = want_map
    want = oracle.run_frame(g)

    d = ft.DeviceFrame(f, "cuda")
    dm = ft.DeviceMap(f["map"], cap)
    dm.edit(ctx, remove, other)
    d.map = dm.struct                      # the frame's search reads the edited device map
    d.nM = dm.n
    for v in d.views:                      # outputs sized for the edited map
        for k in ("mp_match", "mp_dist"):
            v["out_t"][k] = torch.empty(dm.n, dtype=torch.int32, device="cuda")
        o = v["out_t"]
        v["out"] = ft.ft_search_out(ft._ptr(o["mp_match"]), ft._ptr(o["mp_dist"]), ft._ptr(o["kp_match"]),
                                    ft._ptr(o["n_matches"]))
    d.run(ctx)
    torch.cuda.synchronize()
    got = d.results()
    for v, (gs, ws) in enumerate(zip(got["search"], want["search"])):
        compare_search(gs, ws, f"[{kind} view {v}]")
