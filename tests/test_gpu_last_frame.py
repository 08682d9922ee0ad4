"""Device last-frame search by projection (ft_search_last_frame) against the
CPU oracle, element by element.

Cases: the pinhole frame with its stereo right coordinates, both fisheye
views (Kannala-Brandt projection in binary64), the clustered scene (3000
keypoints in hot cells) and tiny frames (ragged tiles); the three directions
of motion; with and without the rotation check; empty inputs; bad parameters.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(ft):
    return ft.Context(ft.default_limits(max_batch_frames=1, max_map_points=32768, max_inflight=1))


def _run(ft, ctx, case):
    d = ft.DeviceLastFrame(case, "cuda")
    d.run(ctx)
    torch.cuda.synchronize()
    return d.results()


def _compare(got, want, tag):
    for k in ("last_match", "last_dist", "kp_match"):
        bad = np.nonzero(got[k] != want[k])[0]
        assert bad.size == 0, f"{tag} {k}: {bad.size} differ, first {bad[:5].tolist()}"
    assert got["n_matches"] == want["n_matches"], tag


FRAMES = {"pinhole": lambda: synth.pinhole_frame_1200()[0], "fisheye": lambda: synth.fisheye_frame_1500()[0],
          "clustered": lambda: synth.clustered_search_20000()[0]}


@pytest.mark.parametrize("direction", [0, 1, -1])
@pytest.mark.parametrize("kind", ["pinhole", "fisheye", "clustered"])
def test_last_frame_full_size(ft, ctx, kind, direction):
    f = FRAMES[kind]()
    for view in range(len(f["search"])):
        for rot in (1, 0):
            case = synth.last_frame_case(f, 950 + view, direction=direction, view=view, check_orientation=rot)
            say(kind, "view", view, "direction", direction, "rotation check", rot, "points", len(case["last"]["octave"]))
            want = oracle.search_last_frame(case)
            _compare(_run(ft, ctx, case), want, f"{kind}/{view}/{direction}/{rot}")


@pytest.mark.parametrize("seed", [961, 962, 963])
def test_last_frame_tiny(ft, ctx, seed):
    for f in (synth.tiny_pinhole(seed), synth.tiny_fisheye(seed), synth.tiny_clustered(seed)):
        case = synth.last_frame_case(f, seed, direction=seed % 3 - 1)
        say("tiny", f["kind"], seed)
        _compare(_run(ft, ctx, case), oracle.search_last_frame(case), f"tiny {f['kind']} {seed}")


def test_last_frame_empty_inputs(ft, ctx):
    f = synth.tiny_pinhole(971)
    case = synth.last_frame_case(f, 971)
    none = dict(case, last={k: v[:0] for k, v in case["last"].items()})
    got = _run(ft, ctx, none)
    assert (got["kp_match"] == -1).all() and got["n_matches"] == 0 and got["last_match"].size == 0
    nokp = dict(case, kps={k: v[:0] for k, v in case["kps"].items()}, u_right=None, preassigned=None)
    got = _run(ft, ctx, nokp)
    assert (got["last_match"] == -1).all() and (got["last_dist"] == -1).all() and got["n_matches"] == 0


def test_last_frame_rejects_bad_parameters(ft, ctx):
    f = synth.tiny_pinhole(972)
    case = synth.last_frame_case(f, 972)
    d = ft.DeviceLastFrame(case, "cuda")
    for field, value in (("direction", 2), ("bins", 0), ("bins", 65), ("th_high", 300), ("th", 0.0)):
        old = getattr(d.params, field)
        setattr(d.params, field, value)
        assert d.run(ctx, check=False) == ft.FT_ERR_INVALID_ARGUMENT, field
        setattr(d.params, field, old)
    torch.cuda.synchronize()
    assert int(d.o["n_matches"][0]) == -7          # nothing was enqueued
