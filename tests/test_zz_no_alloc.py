"""The allocation-free search entry point against the context's search.

ft_search_local_points_noalloc runs the search with its workspace in a fixed
device array instead of a context's arena.  Two calls in a row (the second on a
smaller frame, so the array holds the larger call's leftovers) must give
exactly the outputs of ft_search_local_points and leave the device's free
memory unchanged, and sizes beyond the array's limits must be rejected before
anything runs.
"""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ft():
    from paper_2509_10757_amd import binding
    return binding


def _outputs(ft, dframe, view):
    i32 = dict(dtype=torch.int32, device="cuda")
    t = {"mp_match": torch.full((dframe.nM,), -5, **i32), "mp_dist": torch.full((dframe.nM,), -5, **i32),
         "kp_match": torch.full((view["kps"].n,), -5, **i32), "n_matches": torch.full((1,), -5, **i32)}
    s = ft.ft_search_out(*(ft._ptr(t[k]) for k in ("mp_match", "mp_dist", "kp_match", "n_matches")))
    return t, s


def _ur(ft, dframe, view):
    return ft._ptr(dframe.o["u_right"]) if view["use_u_right"] else None


def test_noalloc_search_equals_context_search(ft):
    ctx = ft.Context(ft.default_limits(max_batch_frames=1, max_map_points=32768, max_inflight=1))
    big = synth.clustered_search_20000()[0]          # 20000 map points, 3000 keypoints, 96x64 grid
    small = synth.pinhole_frame_1200()[0]            # 3000 map points, 1200 keypoints, u_right gate
    # the first call in a process maps the library's scratch array on this
    # device (once, kept until exit); no call after it may allocate
    warm = synth.tiny_clustered(933)
    dw = ft.DeviceFrame(warm, "cuda")
    vw = dw.views[0]
    _, sw = _outputs(ft, dw, vw)
    ft.ft_search_local_points_noalloc(dw.map, vw["cam"], vw["kps"].struct(), None, ft._ptr(vw["pre_t"]),
                                      vw["grid"], dw.scales, dw.search_params, sw)
    torch.cuda.synchronize()
    for name, f in (("clustered 20000/3000", big), ("pinhole 3000/1200", small)):
        say("noalloc search on", name)
        d = ft.DeviceFrame(f, "cuda")
        d.run(ctx)                                   # stereo outputs (u_right) + context search
        torch.cuda.synchronize()
        for vi, v in enumerate(d.views):
            want = {k: t.cpu().numpy() for k, t in v["out_t"].items()}
            t, s = _outputs(ft, d, v)
            torch.cuda.synchronize()
            free0, _ = torch.cuda.mem_get_info()
            ft.ft_search_local_points_noalloc(d.map, v["cam"], v["kps"].struct(), _ur(ft, d, v),
                                              ft._ptr(v["pre_t"]), v["grid"], d.scales, d.search_params, s)
            torch.cuda.synchronize()
            free1, _ = torch.cuda.mem_get_info()
            assert free1 == free0, (name, vi, free0, free1)   # the call allocated nothing
            got = {k: x.cpu().numpy() for k, x in t.items()}
            for k in want:
                assert np.array_equal(got[k], want[k]), (name, vi, k)
            say(" view", vi, "matches", int(got["n_matches"][0]))
            assert got["n_matches"][0] > 0


def test_noalloc_rejects_sizes_beyond_its_array(ft):
    f = synth.clustered_search_20000()[0]
    d = ft.DeviceFrame(f, "cuda")
    v = d.views[0]
    t, s = _outputs(ft, d, v)
    torch.cuda.synchronize()
    too_many_map = ft.ft_map_points.from_buffer_copy(d.map)
    too_many_map.n = ft.FT_NOALLOC_MAX_MAP + 1
    st = ft.ft_search_local_points_noalloc(too_many_map, v["cam"], v["kps"].struct(), None, None, v["grid"],
                                           d.scales, d.search_params, s, check=False)
    assert st == ft.FT_ERR_CAPACITY
    assert b"max_map_points" in ft.load().ft_last_error(None)
    kps = v["kps"].struct()
    kps.n = ft.FT_NOALLOC_MAX_KP + 1
    st = ft.ft_search_local_points_noalloc(d.map, v["cam"], kps, None, None, v["grid"], d.scales,
                                           d.search_params, s, check=False)
    assert st == ft.FT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert int(t["n_matches"][0]) == -5                # nothing was enqueued
