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


def _host_points(ctx, pts):
    """The five arrays of `pts` packed into one ft_host_alloc block."""
    import ctypes as ct
    keys = ("pos", "normal", "dmin", "dmax", "desc")
    sizes = [-(-pts[k].nbytes // 256) * 256 for k in keys]
    base = ctx.ft_host_alloc(max(sum(sizes), 256))
    view = np.ctypeslib.as_array((ct.c_uint8 * max(sum(sizes), 256)).from_address(base))
    addr, at = [], 0
    for k, sz in zip(keys, sizes):
        view[at:at + pts[k].nbytes] = np.ascontiguousarray(pts[k]).view(np.uint8).reshape(-1)
        addr.append(base + at)
        at += sz
    return base, addr


def test_inserts_read_from_pinned_host_memory(ft, ctx):
    """Inserted points in an ft_host_alloc block (read by the append kernel
    over the bus) give the same map as the oracle; arrays only partly in host
    blocks are rejected with the map unchanged."""
    mp = _points(3000, 41, 0)
    cap = 4000
    dm = ft.DeviceMap(mp, cap)
    rng = np.random.default_rng(42)
    tag = 50000
    for step in range(6):
        n = dm.n
        remove = rng.choice(n, int(rng.integers(0, 300)), replace=False).tolist()
        m = int(rng.integers(1, 300))
        ins = _points(m, 300 + step, tag)
        tag += m
        base, addr = _host_points(ctx, ins)
        want = oracle.map_update(mp, cap, remove, ins)
        ctx.ft_map_update(dm.struct, cap, remove, ft.ft_map_points(m, *addr))
        torch.cuda.synchronize()
        ctx.ft_host_free(base)
        _same(dm.host(), want, step)
        mp = want
    # one array on the device, the others in a host block: rejected
    ins = _points(10, 77, tag)
    base, addr = _host_points(ctx, ins)
    dev_dmin = torch.from_numpy(ins["dmin"]).cuda()
    bad = ft.ft_map_points(10, addr[0], addr[1], dev_dmin.data_ptr(), addr[3], addr[4])
    n = dm.n
    assert ctx.ft_map_update(dm.struct, cap, [], bad, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    # a host array running past the end of its block: rejected
    short = ft.ft_map_points(10, addr[0], addr[1], addr[2], addr[3], addr[4] + 256 - 16)
    assert ctx.ft_map_update(dm.struct, cap, [], short, check=False) == ft.FT_ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
    ctx.ft_host_free(base)
    assert dm.n == n
    _same(dm.host(), mp, "unchanged")


def test_many_edits_in_flight_behind_a_busy_stream(ft, ctx):
    """More edits enqueued back to back, behind other work on their stream,
    than the pair staging has events for: staging is reused only after the
    edit that held it has ended, so every edit lands as the oracle's."""
    mp0 = _points(2000, 51, 0)
    cap = 2600
    dm = ft.DeviceMap(mp0, cap)
    rng = np.random.default_rng(52)
    edits, mp, tag, n = [], mp0, 70000, 2000
    for step in range(150):
        remove = rng.choice(n, int(rng.integers(0, 40)), replace=False).tolist()
        m = min(int(rng.integers(0, 40)), cap - (n - len(remove)))
        ins = _points(m, 400 + step, tag)
        tag += m
        mp = oracle.map_update(mp, cap, remove, ins)
        n = len(mp["dmin"])
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in ins.items()} if m else None
        edits.append((remove, m, dev))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(4):
            a = a @ a * 1e-3              # work the edits queue behind
    for remove, m, dev in edits:
        pts = ft.ft_map_points(m, *(ft._ptr(dev[k]) for k in ("pos", "normal", "dmin", "dmax", "desc"))) \
            if m else None
        ctx.ft_map_update(dm.struct, cap, remove, pts, stream=s)
    s.synchronize()
    assert dm.n == n
    _same(dm.host(), mp, "after 150 queued edits")
