"""Serving streams whose local maps change every frame (Update Local Map's
output, Section II-D, kept on the device): the executor edits each stream's
device map in place before the frame's batch (ft_map_update), frames of one
stream run one at a time and in order, every served frame equals the
oracle's result over the oracle's own edited map, and the device maps and the
executor's slot record end equal to the oracle's."""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.serving import make_streams, poisson_arrivals
from tests.parity import compare_frame

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_maps(s, last_seq):
    """The stream's map at every sequence number 0..last_seq by the oracle's
    edit rule, and the point id of each slot at the end (from a second map
    edited alongside whose dmin holds the point ids)."""
    pts = s["points"]
    ids0 = np.asarray(s["map_ids0"])
    tag_all = dict(pts)
    tag_all["dmin"] = np.arange(len(pts["dmin"]), dtype=np.float32)   # ids < 2**24: exact
    mp = {k: v[ids0] for k, v in pts.items()}
    tag = {k: v[ids0] for k, v in tag_all.items()}
    cap = len(ids0)
    maps = [mp]
    for k in range(1, last_seq + 1):
        e = s["edits"][k % len(s["frames"])]
        slot = {int(p): i for i, p in enumerate(tag["dmin"].astype(np.int64))}
        rem = [slot[int(p)] for p in e["remove_ids"]]
        mp = oracle.map_update(mp, cap, rem, {kk: v[e["insert_ids"]] for kk, v in pts.items()})
        tag = oracle.map_update(tag, cap, rem, {kk: v[e["insert_ids"]] for kk, v in tag_all.items()})
        assert mp is not None and tag is not None
        maps.append(mp)
    return maps, tag["dmin"].astype(np.int64)


def test_served_frames_follow_their_edited_maps(ft):
    from paper_2509_10757_amd.serve import DeviceExecutor, Scheduler
    streams = make_streams(np.random.SeedSequence(57), n_streams=6, frames_per_stream=3, world_points=200_000,
                           map_range=(2000, 8000), kp_range=(500, 1200), map_churn=0.05)
    ex = DeviceExecutor(streams, max_batch=16, max_inflight=2)
    served = []

    def keep(h):
        _, slots, frames = ex.handles[h]
        for slot, fr in zip(slots, frames):
            s = streams[fr.stream]
            f = s["frames"][fr.seq % len(s["frames"])]
            served.append(((fr.stream, fr.seq),
                           ex.results(slot, f["kind"], len(f["left"]["x"]), s["n_map"], len(f["search"]),
                                      sync=False)))
    sch = Scheduler(ex, hbm_budget=1 << 32, max_batch=16, max_inflight=2, sequential=True)
    for s in streams:
        assert sch.register_stream(s["id"], ex.footprint(s["id"]))
    arr = poisson_arrivals(np.random.default_rng(4), streams, 0.35, speedup=1.0)
    last = {}
    for _, sid, seq in arr:
        last[sid] = max(last.get(sid, 0), seq)
    assert all(last[s["id"]] >= len(s["frames"]) for s in streams), "every stream's pool wraps at least once"
    say("arrivals", len(arr), "last sequence numbers", last)
    ex.on_release = keep
    try:
        st = sch.run(arr).summary()
    finally:
        ex.on_release = None
    say({k: v for k, v in st.items() if k != "rejected_streams"})
    assert st["frames"] == len(arr) and st["failed"] == 0
    assert len(served) == len(arr)
    maps = {sid: _oracle_maps(streams[sid], last[sid]) for sid in last}
    for (sid, seq), got in served:
        s = streams[sid]
        f = dict(s["frames"][seq % len(s["frames"])])
        f["map"] = maps[sid][0][seq]
        compare_frame(got, oracle.run_frame(f))
    torch.cuda.synchronize()
    for sid, (mlist, ids) in maps.items():
        assert np.array_equal(ex.id_rec[sid]["slot_id"][:len(ids)], ids), sid
        assert np.array_equal(np.sort(np.flatnonzero(ex.id_rec[sid]["slot_of"] >= 0)), np.sort(ids)), sid
        assert ex.map_struct[sid].n == len(ids)
        for k, v in ex.maps[sid].items():
            assert np.array_equal(v.cpu().numpy().view(np.uint8), mlist[-1][k].view(np.uint8)), (sid, k)
