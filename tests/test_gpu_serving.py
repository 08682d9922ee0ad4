"""Serving on the GPU: a frame gives the same result alone and in a mixed
batch (bit-identical, and equal to the oracle), and a short real-time run
serves every arrival."""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth.serving import make_streams
from tests.parity import bit_equal, compare_frame

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def streams():
    return make_streams(np.random.SeedSequence(55), n_streams=6, frames_per_stream=2,
                        world_points=200_000, map_range=(2000, 12000), kp_range=(500, 1500))


@pytest.fixture(scope="module")
def executor(streams):
    from paper_2509_10757_amd.serve import DeviceExecutor
    ex = DeviceExecutor(streams, max_batch=16, max_inflight=2)
    for s in streams:
        ex.admit(s["id"])
    return ex


def _wait(ex, h):
    while not ex.done(h):
        pass


def _result(ex, h, streams, idx):
    _, slots, frames = ex.handles[h]
    fr = frames[idx]
    s = streams[fr.stream]
    f = s["frames"][fr.seq % len(s["frames"])]
    return ex.results(slots[idx], f["kind"], len(f["left"]["x"]), len(f["map"]["dmin"]),
                      len(f["search"])), f


def test_result_alone_equals_result_in_mix(streams, executor):
    from paper_2509_10757_amd.serve import Frame
    ex = executor
    mix = [Frame(s["id"], q, 0.0) for q in range(2) for s in streams]
    say("mix of", len(mix))
    h = ex.launch(mix)
    _wait(ex, h)
    in_mix = [_result(ex, h, streams, i) for i in range(len(mix))]
    ex.release(h)
    for i, fr in enumerate(mix):
        h1 = ex.launch([fr], per_frame=True)      # the same frame alone, single-frame calls
        _wait(ex, h1)
        alone, f = _result(ex, h1, streams, 0)
        ex.release(h1)
        bit_equal(alone, in_mix[i][0])
        compare_frame(in_mix[i][0], oracle.run_frame(f))


def test_short_real_time_run_serves_everything(streams, executor):
    """Continuous batching in real time with batches overlapping on the
    device: every arrival is served, and every served frame's outputs (copied
    when its batch ends, before its slots are reused) equal the oracle's."""
    from paper_2509_10757_amd.serve import Scheduler
    from synth.serving import poisson_arrivals
    served = []

    def keep(h):
        _, slots, frames = executor.handles[h]
        for slot, fr in zip(slots, frames):
            s = streams[fr.stream]
            f = s["frames"][fr.seq % len(s["frames"])]
            served.append(((fr.stream, fr.seq % len(s["frames"])),
                           executor.results(slot, f["kind"], len(f["left"]["x"]), len(f["map"]["dmin"]),
                                            len(f["search"]), sync=False)))
    sch = Scheduler(executor, hbm_budget=1 << 32, max_batch=16, max_inflight=2)
    for s in streams:
        sch.register_stream(s["id"], executor.footprint(s["id"]))
    arr = poisson_arrivals(np.random.default_rng(3), streams, 1.0, speedup=16.0)
    executor.on_release = keep
    try:
        st = sch.run(arr).summary()
    finally:
        executor.on_release = None
    say({k: v for k, v in st.items() if k != "rejected_streams"})
    assert st["frames"] == len(arr) and st["failed"] == 0
    assert st["p99_ms"] < 1000.0
    assert st["max_overlap"] >= 2, "no two batches were ever in flight together"
    assert len(served) == len(arr)
    want = {}
    for key, got in served:
        if key not in want:
            sid, q = key
            want[key] = oracle.run_frame(streams[sid]["frames"][q])
        compare_frame(got, want[key])


def test_evicted_stream_frees_its_device_memory(streams, executor):
    """Eviction frees exactly the bytes the stream's footprint counts, and the
    stream can be admitted again."""
    sid = next(s["id"] for s in streams if s["kind"] == "pinhole")
    before = executor.resident_bytes()
    executor.evict(sid)
    assert before - executor.resident_bytes() == executor.footprint(sid)
    executor.admit(sid)
    assert executor.resident_bytes() == before


def test_admission_rejects_streams_beyond_budget(streams, executor):
    from paper_2509_10757_amd.serve import Scheduler
    fp = [executor.footprint(s["id"]) for s in streams]
    sch = Scheduler(executor, hbm_budget=sum(fp[:3]), max_batch=16, max_inflight=2)
    ok = [sch.register_stream(s["id"], f) for s, f in zip(streams, fp)]
    assert ok[:3] == [True] * 3 and not all(ok[3:])
    torch.cuda.synchronize()
