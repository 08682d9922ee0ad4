"""Device path (through the C ABI) against the CPU oracle, element by element.

Sizes: tiny frames (several tiles and ragged tails) for every kind, the full
single-frame workloads (pinhole 1200 kp / 3000 map points, fisheye 1500 kp /
5000 map points, clustered 3000 kp / 20000 map points), the 64-frame batched
workload as it is benchmarked, a maximum-size frame, and degenerate cases.
"""
import copy
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity import bit_equal, compare_frame

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(ft):
    return ft.Context(ft.default_limits(max_batch_frames=64, max_map_points=65536))


def run_device(ft, ctx, frame, batch=False):
    df = ft.DeviceFrame(frame, "cuda")
    if batch:
        t = ctx.ft_batch_submit([df.job()])
        ctx.ft_batch_wait(t)
    else:
        df.run(ctx)
    torch.cuda.synchronize()
    return df.results()


@pytest.mark.parametrize("seed", [101, 102, 103, 104, 105])
def test_tiny_pinhole(ft, ctx, seed):
    f = synth.tiny_pinhole(seed, n_kp=int(60 + 37 * (seed % 5)), n_map=200 + seed)
    say("tiny pinhole", seed)
    compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


@pytest.mark.parametrize("seed", [201, 202, 203, 204, 205])
def test_tiny_fisheye(ft, ctx, seed):
    f = synth.tiny_fisheye(seed, n_kp=int(70 + 41 * (seed % 5)), n_map=150 + seed)
    say("tiny fisheye", seed)
    compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


@pytest.mark.parametrize("seed", [301, 302, 303])
def test_tiny_clustered(ft, ctx, seed):
    f = synth.tiny_clustered(seed, n_map=300 + 111 * (seed % 3), n_kp=97 + seed % 7)
    say("tiny clustered", seed)
    compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


@pytest.mark.parametrize("name", sorted(synth.SINGLE_FRAME))
def test_full_size_single_frame(ft, ctx, name):
    f = synth.workload(name)[0]
    say("workload", name)
    got = run_device(ft, ctx, f)
    compare_frame(got, oracle.run_frame(f))
    assert got["search"][0]["n_matches"] > 100


def test_batched_workload_matches_oracle_and_single_frame_path(ft, ctx):
    frames = synth.mixed_batch()
    say("batched workload: 64 frames")
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    t = ctx.ft_batch_submit([d.job() for d in dfs])
    ctx.ft_batch_wait(t)
    torch.cuda.synchronize()
    batch = [d.results() for d in dfs]
    for f, got in zip(frames, batch):
        compare_frame(got, oracle.run_frame(f))
    # the same frames through the single-frame calls give identical bits
    for f, b in zip(frames[:8], batch[:8]):
        bit_equal(run_device(ft, ctx, f), b)


def test_repeat_runs_are_bit_identical(ft, ctx):
    f = synth.clustered_search_20000()[0]
    first = run_device(ft, ctx, f)
    for _ in range(4):
        bit_equal(run_device(ft, ctx, f), first)
    f = synth.fisheye_frame_1500()[0]
    first = run_device(ft, ctx, f, batch=True)
    for _ in range(3):
        bit_equal(run_device(ft, ctx, f, batch=True), first)


def test_maximum_size_frame(ft, ctx):
    f = synth.pinhole.pinhole_frame(np.random.SeedSequence(4242), n_kp=4096, n_map=65536)
    say("max size frame")
    compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


# ------------------------------------------------------------ degenerate cases
def _empty_kps():
    return {"x": np.zeros(0, np.float32), "y": np.zeros(0, np.float32),
            "octave": np.zeros(0, np.uint8), "desc": np.zeros((0, 32), np.uint8)}


def _drop_preassigned(f, n):
    for s in f["search"]:
        s["preassigned"] = np.zeros(n, np.uint8)


@pytest.mark.parametrize("maker", [synth.tiny_pinhole, synth.tiny_fisheye])
def test_empty_left_and_right(ft, ctx, maker):
    for side in ("left", "right"):
        f = maker(501)
        f[side] = _empty_kps()
        for s in f["search"]:
            if s["image"] == side:
                s["preassigned"] = np.zeros(0, np.uint8)
        say("empty", side, f["kind"])
        compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


def test_empty_map(ft, ctx):
    for maker in (synth.tiny_pinhole, synth.tiny_fisheye, synth.tiny_clustered):
        f = maker(502)
        f["map"] = {k: v[:0] for k, v in f["map"].items()}
        compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


def test_fisheye_fewer_than_two_targets(ft, ctx):
    f = synth.tiny_fisheye(503, n_kp=100)
    xs = np.sort(f["right"]["x"])
    f["stereo_cam"]["overlap_right"] = np.array([xs[0], xs[0]], np.float32)  # exactly one target
    want = oracle.run_frame(f)
    assert want["stereo"]["stats"]["T"] == 1 and want["stereo"]["n_matches"] == 0
    compare_frame(run_device(ft, ctx, f), want)


def test_grid_shapes_and_far_keypoints(ft, ctx):
    base = synth.tiny_clustered(504)
    for grid in [(1, 1), (3, 97), (128, 64)]:
        f = copy.deepcopy(base)
        f["search"][0]["grid"] = grid
        f["left"]["x"][::17] = np.float32(1e6)       # far outside the image
        f["left"]["y"][::23] = np.float32(-50.0)
        say("grid", grid)
        compare_frame(run_device(ft, ctx, f), oracle.run_frame(f))


def test_all_preassigned_and_no_u_right_gate(ft, ctx):
    f = synth.tiny_pinhole(505)
    f["search"][0]["preassigned"][:] = 1
    got = run_device(ft, ctx, f)
    want = oracle.run_frame(f)
    compare_frame(got, want)
    assert want["search"][0]["n_matches"] == 0
    f = synth.tiny_pinhole(506)
    f["search"][0]["use_u_right"] = False
    compare_frame(run_device(ft, ctx, f),
                  {"kind": "pinhole", "stereo": oracle.stereo_pinhole(f),
                   "search": [oracle.search_local_points(f, 0)]})


def test_all_keypoints_identical_descriptor_ties(ft, ctx):
    """Every descriptor equal: all distances tie, so indices alone decide."""
    f = synth.tiny_clustered(507)
    f["left"]["desc"][:] = f["left"]["desc"][0]
    f["map"]["desc"][:] = f["left"]["desc"][0]
    f2 = synth.tiny_fisheye(508)
    f2["left"]["desc"][:] = f2["left"]["desc"][0]
    f2["right"]["desc"][:] = f2["left"]["desc"][0]
    for fr in (f, f2):
        compare_frame(run_device(ft, ctx, fr), oracle.run_frame(fr))


# ------------------------------------------------------------------ errors
def test_invalid_arguments_enqueue_nothing(ft, ctx):
    f = synth.tiny_pinhole(601)
    df = ft.DeviceFrame(f, "cuda")
    df.o["right_idx"].fill_(12345)
    bad = ft.ft_scales.from_buffer_copy(df.scales)
    bad.n_levels = 7
    st = ctx.ft_stereo_match_pinhole(df.left.struct(), df.right.struct(), df.pyr_left, df.pyr_right,
                                     bad, df.stereo_cam, df.stereo_params, df.stereo_out, check=False)
    assert st == ft.FT_ERR_INVALID_ARGUMENT
    params = ft.ft_pinhole_params.from_buffer_copy(df.stereo_params)
    params.band = 100.0
    st = ctx.ft_stereo_match_pinhole(df.left.struct(), df.right.struct(), df.pyr_left, df.pyr_right,
                                     df.scales, df.stereo_cam, params, df.stereo_out, check=False)
    assert st == ft.FT_ERR_INVALID_ARGUMENT
    big = df.left.struct()
    big.n = ctx.limits.max_kp_per_image + 1
    st = ctx.ft_stereo_match_pinhole(big, df.right.struct(), df.pyr_left, df.pyr_right, df.scales,
                                     df.stereo_cam, df.stereo_params, df.stereo_out, check=False)
    assert st == ft.FT_ERR_CAPACITY
    grid = ft.ft_grid(200, 100)
    v = df.views[0]
    st = ctx.ft_search_local_points(df.map, v["cam"], v["kps"].struct(), None, None, grid, df.scales,
                                    df.search_params, v["out"], check=False)
    assert st == ft.FT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert bool((df.o["right_idx"] == 12345).all())
    # the context is still usable after rejected calls
    df.run(ctx)
    torch.cuda.synchronize()
    compare_frame(df.results(), oracle.run_frame(f))


def test_batch_tickets_poll_and_wait(ft, ctx):
    frames = [synth.tiny_pinhole(700 + i) for i in range(3)] + [synth.tiny_fisheye(710 + i) for i in range(3)]
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    t1 = ctx.ft_batch_submit([d.job() for d in dfs[:3]])
    t2 = ctx.ft_batch_submit([d.job() for d in dfs[3:]])
    assert t1 != t2
    ctx.ft_batch_wait(t2)
    assert ctx.ft_batch_poll(t1) and ctx.ft_batch_poll(t2)
    for f, d in zip(frames, dfs):
        compare_frame(d.results(), oracle.run_frame(f))


# ------------------------------------------------------- launch shapes / tuner
def test_lane_groups_do_not_change_results(ft, ctx):
    frames = synth.mixed_batch(n_frames=8)
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    jobs = [d.job() for d in dfs]
    ref = None
    try:
        for shape in [(1, 1, 1024), (2, 16, 256), (4, 8, 256), (8, 4, 1024), (16, 2, 1024), (8, 1, 256)]:
            ctx.ft_set_shapes(*shape)
            say("shapes", shape)
            ctx.ft_batch_wait(ctx.ft_batch_submit(jobs))
            torch.cuda.synchronize()
            res = [d.results() for d in dfs]
            if ref is None:
                ref = res
                for f, r in zip(frames, res):
                    compare_frame(r, oracle.run_frame(f))
            else:
                for a, b in zip(res, ref):
                    bit_equal(a, b)
    finally:
        ctx.ft_set_shapes(8, 1)


def test_autotune_picks_valid_shapes_and_caches(ft, ctx, tmp_path):
    frames = synth.mixed_batch(n_frames=6)
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    jobs = [d.job() for d in dfs]
    cache = str(tmp_path / "shapes.jsonl")
    try:
        chosen = ctx.ft_autotune(jobs, cache)
        assert chosen[0] in (1, 2, 4, 8, 16) and chosen[1] in (1, 2, 4, 8, 16)
        assert chosen[2] in (256, 1024)
        text = open(cache).read()
        assert '"best_lanes": %d' % chosen[0] in text
        ctx.ft_set_shapes(1, 1, 1024 + 256 - chosen[2])
        assert ctx.ft_autotune(jobs, cache) == chosen        # served from the cache
        assert ctx.ft_get_shapes() == chosen
        assert open(cache).read() == text
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs))
        torch.cuda.synchronize()
        for f, d in zip(frames, dfs):
            compare_frame(d.results(), oracle.run_frame(f))
    finally:
        ctx.ft_set_shapes(8, 1)


def test_graph_replays_match_eager(ft, ctx):
    frames = synth.mixed_batch(n_frames=8)
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    jobs = [d.job() for d in dfs]
    try:
        ctx.ft_set_exec_mode(ft.FT_EXEC_EAGER)
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs))
        torch.cuda.synchronize()
        ref = [d.results() for d in dfs]
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs[:5]))
        torch.cuda.synchronize()
        ref5 = [d.results() for d in dfs[:5]]
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
        for rep in range(4):
            for d in dfs:                                   # eager work between replays
                for t in d.o.values():
                    t.fill_(-7)
                for v in d.views:
                    for t in v["out_t"].values():
                        t.fill_(-9)
            torch.cuda.synchronize()
            sub = jobs if rep % 2 == 0 else jobs[:5]
            ctx.ft_batch_wait(ctx.ft_batch_submit(sub))
            torch.cuda.synchronize()
            want = ref if rep % 2 == 0 else ref5
            for d, w in zip(dfs, want):
                bit_equal(d.results(), w)
    finally:
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)


def _clobber(dfs):
    for d in dfs:
        for t in d.o.values():
            t.fill_(-7)
        for v in d.views:
            for t in v["out_t"].values():
                t.fill_(-9)
    torch.cuda.synchronize()


def test_graph_nodes_follow_every_batch_shape(ft, ctx):
    """The lane's one instantiated graph serves batches of every shape: each
    submission sets the table size and every phase's grid in place.  Batches
    with phases that have no tiles (pinhole only, fisheye only, search only),
    of one frame and of all frames, and the same batches after a shape change
    (which rebuilds the graphs) give the eager results; eager work runs
    between the replays."""
    frames = synth.mixed_batch(n_frames=12)
    dfs = [ft.DeviceFrame(f, "cuda") for f in frames]
    jobs = [d.job() for d in dfs]
    pin = [k for k, f in enumerate(frames) if f["kind"] == "pinhole"]
    fish = [k for k, f in enumerate(frames) if f["kind"] == "fisheye"]
    assert pin and fish
    search_only = [dfs[k].job(stereo=False) for k in fish[:2]]
    subsets = [list(range(12)), pin, fish, [0], list(range(12)), fish[:1], pin[:3]]
    try:
        ctx.ft_set_exec_mode(ft.FT_EXEC_EAGER)
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs))
        torch.cuda.synchronize()
        ref = [d.results() for d in dfs]
        ctx.ft_batch_wait(ctx.ft_batch_submit(search_only))
        torch.cuda.synchronize()
        ref_search = [dfs[k].results()["search"] for k in fish[:2]]
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
        for shapes in ((8, 1), (4, 2, 256)):
            ctx.ft_set_shapes(*shapes)
            for sub in subsets:
                say("shapes", shapes, "graph batch of frames", sub)
                _clobber(dfs)
                ctx.ft_batch_wait(ctx.ft_batch_submit([jobs[k] for k in sub]))
                torch.cuda.synchronize()
                for k in sub:
                    bit_equal(dfs[k].results(), ref[k])
            say("shapes", shapes, "graph batch of search-only jobs")
            _clobber(dfs)
            ctx.ft_batch_wait(ctx.ft_batch_submit(search_only))
            torch.cuda.synchronize()
            for k, w in zip(fish[:2], ref_search):
                for a, b in zip(dfs[k].results()["search"], w):
                    for key in a:
                        assert np.array_equal(a[key], b[key]), key
    finally:
        ctx.ft_set_shapes(8, 1)
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)


@pytest.mark.parametrize("half_win,half_range", [(3, 7), (5, 9), (2, 2)])
def test_refinement_window_sizes(ft, ctx, half_win, half_range):
    """Windows other than 11x11 / +-5 take the one-wave-per-match refinement;
    single-frame and batched results equal the oracle."""
    f = synth.pinhole_frame_1200()[0]
    f["stereo_params"] = dict(f["stereo_params"], half_win=half_win, half_range=half_range)
    say("refinement window", half_win, half_range)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, ctx, f), want)
    compare_frame(run_device(ft, ctx, f, batch=True), want)


@pytest.mark.parametrize("band", [0.5, 8.0])
def test_epipolar_band_widths(ft, ctx, band):
    """Narrow and wide epipolar bands (the row index scans row_reach bins on
    each side): single-frame and batched results, both best-match blocks,
    equal the oracle."""
    f = synth.pinhole_frame_1200()[0]
    f["stereo_params"] = dict(f["stereo_params"], band=band)
    say("epipolar band", band)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, ctx, f), want)
    try:
        for lanes in (4, 16):
            ctx.ft_set_shapes(lanes, 1)
            compare_frame(run_device(ft, ctx, f, batch=True), want)
    finally:
        ctx.ft_set_shapes(8, 1)


def test_concurrent_batches_on_streams_match(ft):
    """Batches in flight on four streams at once (each its own copy of the
    frames, each its own in-flight lane) give the single-stream results, in
    graph and eager mode."""
    ctx4 = ft.Context(ft.default_limits(max_batch_frames=16, max_map_points=65536, max_inflight=4))
    frames = synth.mixed_batch(n_frames=16)
    copies = [[ft.DeviceFrame(f, "cuda") for f in frames] for _ in range(4)]
    jobs = [[d.job() for d in c] for c in copies]
    streams = [torch.cuda.Stream() for _ in range(4)]
    ctx4.ft_set_exec_mode(ft.FT_EXEC_EAGER)
    ctx4.ft_batch_wait(ctx4.ft_batch_submit(jobs[0]))
    torch.cuda.synchronize()
    ref = [d.results() for d in copies[0]]
    for mode in (ft.FT_EXEC_GRAPH, ft.FT_EXEC_EAGER):
        ctx4.ft_set_exec_mode(mode)
        say("mode", mode)
        for c in copies:
            _clobber(c)
        pending = []
        for rep in range(3):
            for k in range(4):
                if len(pending) >= 4:
                    ctx4.ft_batch_wait(pending.pop(0))
                pending.append(ctx4.ft_batch_submit(jobs[k], streams[k]))
        while pending:
            ctx4.ft_batch_wait(pending.pop(0))
        torch.cuda.synchronize()
        for c in copies:
            for d, w in zip(c, ref):
                bit_equal(d.results(), w)
    ctx4.close()


@pytest.mark.parametrize("level_window", [0, 2, 7])
def test_level_windows(ft, ctx, level_window):
    """The row index is binned per pyramid level and a left keypoint scans only
    the level bins of its window: every window width gives the oracle's
    matches, single-frame and batched."""
    f = synth.pinhole_frame_1200()[0]
    f["stereo_params"] = dict(f["stereo_params"], level_window=level_window)
    say("level window", level_window)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, ctx, f), want)
    compare_frame(run_device(ft, ctx, f, batch=True), want)


def test_tall_row_index_single_level_bin(ft):
    """More rows than the per-level (level, row) histogram holds: the row index
    falls back to one bin for every level and still gives the oracle's matches."""
    tall = ft.Context(ft.default_limits(max_batch_frames=4, max_map_points=65536, max_rows=2048))
    f = synth.pinhole_frame_1200()[0]
    f["stereo_cam"] = dict(f["stereo_cam"], rows=1100)
    say("tall row index")
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, tall, f), want)
    compare_frame(run_device(ft, tall, f, batch=True), want)
    tall.close()


@pytest.mark.parametrize("name", ["fisheye_frame_1500", "clustered_search_20000"])
@pytest.mark.parametrize("lo,hi", [(0, 0), (0, 2), (2, 0), (1, 2)])
def test_search_level_windows(ft, ctx, name, lo, hi):
    """The search's keypoint index holds one bin per predicted level (with the
    octaves of that level's window) when the window spans at most three
    octaves, and one bin for every octave otherwise (1, 2); the fisheye grid is
    merged 2 x 2 and the clustered 96 x 64 grid 3 x 3.  Every window gives the
    oracle's matches, single-frame and batched."""
    f = synth.workload(name)[0]
    f["search_params"] = dict(f["search_params"], level_lo=lo, level_hi=hi)
    say("search level window", name, lo, hi)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, ctx, f), want)
    compare_frame(run_device(ft, ctx, f, batch=True), want)


def test_many_keypoints_single_bin_search_index(ft):
    """24000 keypoints: three level-bin copies of each would exceed the 16-bit
    record offsets, so the search index keeps one bin on the caller's grid and
    still gives the oracle's matches (the keypoints are the clustered frame's
    3000 repeated eight times, copy r with bit 0 of descriptor byte r flipped,
    so near and equal-distance ties abound)."""
    f = synth.clustered_search_20000()[0]
    n, reps = f["left"]["x"].shape[0], 8
    f["left"] = {k: np.concatenate([v] * reps) for k, v in f["left"].items()}
    for r in range(1, reps):
        f["left"]["desc"][r * n:(r + 1) * n, r] ^= 1
    for s in f["search"]:
        s["preassigned"] = np.concatenate([s["preassigned"]] * reps)
    big = ft.Context(ft.default_limits(max_kp_per_image=n * reps, max_map_points=32768, max_batch_frames=2,
                                       max_inflight=1))
    say("many keypoints", n * reps)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, big, f), want)
    compare_frame(run_device(ft, big, f, batch=True), want)
    big.close()


@pytest.mark.parametrize("th_orb", [0, 1, 20])
def test_refinement_list_lengths(ft, ctx, th_orb):
    """The refinement runs over the list of accepted best matches: an empty
    list (threshold 0 accepts nothing), a short one and a longer one give the
    oracle's outputs, single-frame and in a batch beside an unchanged frame."""
    f = synth.pinhole_frame_1200()[0]
    f["stereo_params"] = dict(f["stereo_params"], th_orb=th_orb)
    say("refinement list, th_orb", th_orb)
    want = oracle.run_frame(f)
    compare_frame(run_device(ft, ctx, f), want)
    g = synth.pinhole_frame_1200()[0]
    dfs = [ft.DeviceFrame(f, "cuda"), ft.DeviceFrame(g, "cuda")]
    ctx.ft_batch_wait(ctx.ft_batch_submit([d.job() for d in dfs]))
    torch.cuda.synchronize()
    compare_frame(dfs[0].results(), want)
    compare_frame(dfs[1].results(), oracle.run_frame(g))
