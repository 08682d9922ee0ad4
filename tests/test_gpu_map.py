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


def test_edits_by_point_id_keep_the_slot_record(ft, ctx):
    """Removals named by point id with the library-kept slot record: the map
    equals the oracle's, and the record equals the slot contents of an
    id-tagged map edited by the oracle alongside; invalid ids (out of range,
    not in the map, inserted twice or already present) leave map and record
    unchanged."""
    n_ids, cap = 9000, 5000
    rng = np.random.default_rng(61)
    table = _points(n_ids, 62, 0)                       # dmin = point id: the oracle map is its own tag
    ids0 = np.sort(rng.choice(n_ids, 4000, replace=False))
    mp = {k: v[ids0] for k, v in table.items()}
    dm = ft.DeviceMap(mp, cap)
    slot_id = np.zeros(cap, np.int32)
    slot_id[:len(ids0)] = ids0
    slot_of = np.full(n_ids, -1, np.int32)
    slot_of[ids0] = np.arange(len(ids0))
    rec = ft.ft_map_ids(slot_id.ctypes.data, slot_of.ctypes.data, n_ids)
    for step in range(40):
        live = slot_id[:dm.n].copy()
        rem_ids = rng.choice(live, int(rng.integers(0, min(400, len(live)) + 1)), replace=False)
        free = np.setdiff1d(np.arange(n_ids), live)
        m = min(int(rng.integers(0, 400)), cap - (len(live) - len(rem_ids)), len(free))
        ins_ids = rng.choice(free, m, replace=False)
        # the oracle takes slots: the removed ids' current slots in the oracle's own map
        oracle_slot = {int(v): i for i, v in enumerate(mp["dmin"].astype(np.int64))}
        want = oracle.map_update(mp, cap, [oracle_slot[int(i)] for i in rem_ids],
                                 {k: v[ins_ids] for k, v in table.items()})
        ins = {k: torch.from_numpy(np.ascontiguousarray(v[ins_ids])).cuda() for k, v in table.items()}
        pts = ft.ft_map_points(m, *(ft._ptr(ins[k]) for k in ("pos", "normal", "dmin", "dmax", "desc")))
        ctx.ft_map_update(dm.struct, cap, rem_ids, pts if m else None, ids=rec, insert_ids=ins_ids)
        torch.cuda.synchronize()
        _same(dm.host(), want, step)
        n = dm.n
        assert np.array_equal(slot_id[:n], want["dmin"].astype(np.int32)), step
        assert np.array_equal(np.flatnonzero(slot_of >= 0), np.sort(slot_id[:n])), step
        assert np.array_equal(slot_of[slot_id[:n]], np.arange(n)), step
        mp = want
    live = slot_id[:dm.n].copy()
    free = np.setdiff1d(np.arange(n_ids), live)
    snap = (slot_id.copy(), slot_of.copy(), dm.n)
    one = {k: torch.from_numpy(np.ascontiguousarray(v[:2])).cuda() for k, v in table.items()}
    two = ft.ft_map_points(2, *(ft._ptr(one[k]) for k in ("pos", "normal", "dmin", "dmax", "desc")))
    for rem_ids, ins_ids, what in (([n_ids], [free[0], free[1]], "id out of range"),
                                   ([free[0]], [free[1], free[2]], "removed id not in the map"),
                                   ([], [free[0], free[0]], "inserted twice"),
                                   ([], [live[0], free[0]], "inserted id already in the map"),
                                   ([live[0], live[0]], [free[0], free[1]], "removed twice")):
        st = ctx.ft_map_update(dm.struct, cap, rem_ids, two, ids=rec, insert_ids=ins_ids, check=False)
        assert st == ft.FT_ERR_INVALID_ARGUMENT, what
        assert dm.n == snap[2] and np.array_equal(slot_id, snap[0]) and np.array_equal(slot_of, snap[1]), what
    torch.cuda.synchronize()
    _same(dm.host(), mp, "unchanged")


def test_many_maps_edited_in_one_call(ft, ctx):
    """Rounds of edits of five maps in one ft_map_update_many call each (two
    maps edited by slot, three by point id with their records): every map
    equals the oracle's; an invalid edit among valid ones, or two edits of one
    map, leave every map and record unchanged; an empty call does nothing."""
    rng = np.random.default_rng(71)
    n_ids = 6000
    table = _points(n_ids, 72, 0)
    maps, dms, caps, recs = [], [], [], []
    for k, n0 in enumerate((300, 1200, 2500, 4000, 50)):
        ids0 = np.sort(rng.choice(n_ids, n0, replace=False))
        mp = {key: v[ids0] for key, v in table.items()}
        cap = n0 + 700
        maps.append(mp)
        dms.append(ft.DeviceMap(mp, cap))
        caps.append(cap)
        if k >= 2:
            sid = np.zeros(cap, np.int32)
            sid[:n0] = ids0
            sof = np.full(n_ids, -1, np.int32)
            sof[ids0] = np.arange(n0)
            recs.append((sid, sof, ft.ft_map_ids(sid.ctypes.data, sof.ctypes.data, n_ids)))
        else:
            recs.append(None)
    keep = []

    def edit_for(k):
        dm, mp, cap = dms[k], maps[k], caps[k]
        n = dm.n
        used = set(mp["dmin"].astype(np.int64).tolist())
        nr = int(rng.integers(0, min(300, n) + 1))
        rem_slots = rng.choice(n, nr, replace=False)
        free = np.array(sorted(set(range(n_ids)) - used))
        m = min(int(rng.integers(0, 300)), cap - (n - nr), len(free))
        ins_ids = rng.choice(free, m, replace=False).astype(np.int32)
        want = oracle.map_update(mp, cap, rem_slots, {key: v[ins_ids] for key, v in table.items()})
        dev = {key: torch.from_numpy(np.ascontiguousarray(v[ins_ids])).cuda() for key, v in table.items()}
        pts = ft.ft_map_points(m, *(ft._ptr(dev[key]) for key in ("pos", "normal", "dmin", "dmax", "desc"))) \
            if m else ft.ft_map_points()
        if recs[k] is None:
            rem = np.ascontiguousarray(rem_slots, dtype=np.int32)
            ed = ft.ft_map_edit(nr, rem.ctypes.data if nr else None, pts, None, None)
        else:
            rem = np.ascontiguousarray(mp["dmin"][rem_slots].astype(np.int32))   # the removed points' ids
            ed = ft.ft_map_edit(nr, rem.ctypes.data if nr else None, pts, ins_ids.ctypes.data if m else None,
                                ct.pointer(recs[k][2]))
        keep.extend([rem, ins_ids, dev])
        return ed, want

    import ctypes as ct
    for rnd in range(12):
        order = rng.permutation(5)[: int(rng.integers(1, 6))]
        eds, wants = zip(*[edit_for(int(k)) for k in order])
        torch.cuda.synchronize()
        ctx.ft_map_update_many([dms[k].struct for k in order], [caps[k] for k in order], list(eds))
        torch.cuda.synchronize()
        for k, want in zip(order, wants):
            _same(dms[k].host(), want, (rnd, int(k)))
            maps[k] = want
            if recs[k] is not None:
                n = dms[k].n
                assert np.array_equal(recs[k][0][:n], want["dmin"].astype(np.int32)), (rnd, int(k))
                assert np.array_equal(np.sort(np.flatnonzero(recs[k][1] >= 0)), np.sort(recs[k][0][:n]))
    snap = [(dm.n, None if r is None else (r[0].copy(), r[1].copy())) for dm, r in zip(dms, recs)]
    good, _ = edit_for(0)
    bad_rem = np.array([np.flatnonzero(recs[3][1] < 0)[0]], np.int32)  # an id not in map 3
    bad = ft.ft_map_edit(1, bad_rem.ctypes.data, ft.ft_map_points(), None, ct.pointer(recs[3][2]))
    keep.append(bad_rem)
    assert ctx.ft_map_update_many([dms[0].struct, dms[3].struct], [caps[0], caps[3]], [good, bad],
                                  check=False) == ft.FT_ERR_INVALID_ARGUMENT
    good1, _ = edit_for(1)
    good1b, _ = edit_for(1)
    assert ctx.ft_map_update_many([dms[1].struct, dms[1].struct], [caps[1], caps[1]], [good1, good1b],
                                  check=False) == ft.FT_ERR_INVALID_ARGUMENT
    shared = ft.ft_map_edit(0, None, ft.ft_map_points(), None, ct.pointer(recs[2][2]))
    assert ctx.ft_map_update_many([dms[2].struct, dms[3].struct], [caps[2], caps[3]], [shared, shared],
                                  check=False) == ft.FT_ERR_INVALID_ARGUMENT
    assert ctx.ft_map_update_many([], [], []) == ft.FT_OK
    torch.cuda.synchronize()
    for k, (n, r) in enumerate(snap):
        assert dms[k].n == n
        _same(dms[k].host(), maps[k], ("unchanged", k))
        if r is not None:
            assert np.array_equal(recs[k][0], r[0]) and np.array_equal(recs[k][1], r[1])
