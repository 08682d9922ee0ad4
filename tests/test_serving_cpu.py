"""Serving-loop logic on the CPU with a fake executor and a fake clock:
admission by footprint, FIFO coalescing, in-flight and slot limits, latency
accounting, injected failures, time-outs and stream removal."""
import pytest

from paper_2509_10757_amd.serve import BatchFailed, Frame, Scheduler, ServingStalled


class FakeClock:
    def __init__(self):
        self.t = 100.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch `delay` seconds of fake time after launch."""

    def __init__(self, clock, slots=64, delay=0.002, fail_streams=(), raise_on_launch=False,
                 hang_streams=(), hang_s=None):
        self.clock = clock
        self.slots = slots
        self.delay = delay
        self.fail_streams = set(fail_streams)
        self.hang_streams = set(hang_streams)
        self.hang_s = hang_s          # a hung batch ends after this long (None: never)
        self.evicted = []
        self.raise_on_launch = raise_on_launch
        self.launched = []
        self.h = {}
        self.n = 0
        self.admitted = set()

    def admit(self, sid):
        self.admitted.add(sid)

    def evict(self, sid):
        self.admitted.discard(sid)
        self.evicted.append(sid)

    def free_slots(self):
        return self.slots

    def launch(self, frames, per_frame=False):
        if self.raise_on_launch:
            raise RuntimeError("device lost")
        self.slots -= len(frames)
        self.launched.append([(f.stream, f.seq) for f in frames])
        self.n += 1
        self.h[self.n] = (self.clock() + self.delay, frames)
        return self.n

    def done(self, h):
        t, frames = self.h[h]
        if any(f.stream in self.hang_streams for f in frames):
            return self.hang_s is not None and self.clock() >= t + self.hang_s
        if any(f.stream in self.fail_streams for f in frames):
            raise BatchFailed("kernel error")
        return self.clock() >= t

    def release(self, h):
        _, frames = self.h.pop(h)
        self.slots += len(frames)


def drive(sch, clock, arrivals, dt=0.0005, horizon=1.0):
    """Step the scheduler on fake time."""
    sch.t0 = clock()
    i = 0
    while clock.t - sch.t0 < horizon:
        now = sch.now()
        while i < len(arrivals) and arrivals[i][0] <= now:
            t, s, q = arrivals[i]
            sch.arrive(Frame(s, q, t))
            i += 1
        sch.poll()
        while sch.launch():
            pass
        clock.t += dt
    return sch.stats


def test_admission_by_footprint():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, hbm_budget=100, clock=clock)
    assert sch.register_stream(0, 60)
    assert not sch.register_stream(1, 50)         # would exceed the budget
    assert sch.register_stream(2, 40)
    assert sch.stats.rejected_streams == [1]
    assert ex.admitted == {0, 2}
    sch.remove_stream(0)
    assert sch.register_stream(1, 50)             # room again after removal


def test_fifo_coalescing_and_latency_accounting():
    clock = FakeClock()
    ex = FakeExecutor(clock, delay=0.004)
    sch = Scheduler(ex, hbm_budget=10, max_batch=8, max_inflight=1, clock=clock)
    sch.register_stream(0, 1)
    sch.register_stream(1, 1)
    arrivals = [(0.0001 * k, k % 2, k) for k in range(20)]
    st = drive(sch, clock, arrivals, horizon=0.1)
    assert st.completed == 20 and st.failed == 0
    # first batch launches alone, later ones coalesce up to max_batch, FIFO order kept
    flat = [x for b in ex.launched for x in b]
    assert [q for _, q in flat] == list(range(20))
    assert max(len(b) for b in ex.launched) <= 8
    assert len(ex.launched) < 20
    # latency >= executor delay, and includes queueing behind the batch in flight
    assert min(st.latencies_ms) >= 4.0 - 1e-6
    assert max(st.latencies_ms) > 4.5


def test_inflight_limit_and_slots_respected():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=6, delay=0.01)
    sch = Scheduler(ex, hbm_budget=10, max_batch=4, max_inflight=2, clock=clock)
    sch.register_stream(0, 1)
    arrivals = [(0.0, 0, k) for k in range(30)]
    sch.t0 = clock()
    for t, s, q in arrivals:
        sch.arrive(Frame(s, q, t))
    while sch.launch():
        pass
    assert len(sch.inflight) == 2                 # in-flight limit
    assert sum(len(b) for b in ex.launched) == 6  # slot limit (4 + 2)
    st = drive(sch, clock, [], horizon=0.5)
    assert st.completed == 30


def test_sequential_streams_keep_one_frame_in_flight():
    """Streams with per-frame map edits: a batch holds at most one frame per
    stream, a stream's next frame launches only after its previous frame's
    batch has ended, each stream's frames launch in arrival order, and frames
    of other streams still coalesce."""
    clock = FakeClock()
    ex = FakeExecutor(clock, delay=0.003)
    sch = Scheduler(ex, hbm_budget=10, max_batch=8, max_inflight=3, clock=clock, sequential=True)
    for sid in range(4):
        sch.register_stream(sid, 1)
    arrivals = sorted((0.0002 * k + 0.00001 * sid, sid, k) for sid in range(4) for k in range(6))
    ended = {}
    real_release = ex.release

    def release(h):
        for f in ex.h[h][1]:
            ended[(f.stream, f.seq)] = clock()
        real_release(h)
    ex.release = release
    launched_at = {}
    real_launch = ex.launch

    def launch(frames, per_frame=False):
        for f in frames:
            launched_at[(f.stream, f.seq)] = clock()
        return real_launch(frames, per_frame)
    ex.launch = launch
    st = drive(sch, clock, arrivals, horizon=0.2)
    assert st.completed == 24 and st.failed == 0
    for b in ex.launched:
        assert len({sid for sid, _ in b}) == len(b)
    for sid in range(4):
        seqs = [q for b in ex.launched for s_, q in b if s_ == sid]
        assert seqs == list(range(6))
        for q in range(1, 6):
            assert launched_at[(sid, q)] >= ended[(sid, q - 1)]
    assert max(len(b) for b in ex.launched) > 1


def test_per_frame_mode_never_batches():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, hbm_budget=10, max_batch=64, max_inflight=4, mode="per_frame", clock=clock)
    sch.register_stream(0, 1)
    drive(sch, clock, [(0.0, 0, k) for k in range(10)], horizon=0.2)
    assert all(len(b) == 1 for b in ex.launched)


def test_failures_are_isolated_to_their_batch():
    clock = FakeClock()
    ex = FakeExecutor(clock, fail_streams={1})
    sch = Scheduler(ex, hbm_budget=10, max_batch=1, max_inflight=4, clock=clock)
    for s in (0, 1, 2):
        sch.register_stream(s, 1)
    arrivals = [(0.001 * k, k % 3, k) for k in range(30)]
    st = drive(sch, clock, arrivals, horizon=0.2)
    assert st.failed == 10 and st.completed == 20


def test_launch_exception_fails_the_frames_cleanly():
    clock = FakeClock()
    ex = FakeExecutor(clock, raise_on_launch=True)
    sch = Scheduler(ex, hbm_budget=10, clock=clock)
    sch.register_stream(0, 1)
    st = drive(sch, clock, [(0.0, 0, k) for k in range(5)], horizon=0.05)
    assert st.failed == 5 and st.completed == 0 and not sch.inflight


def test_timeout_marks_batch_failed_but_withholds_its_slots():
    """A batch past its time-out is reported failed at once, but its slots are
    handed out again only after the executor reports its work ended."""
    clock = FakeClock()
    ex = FakeExecutor(clock, hang_streams={7}, hang_s=0.08)
    sch = Scheduler(ex, hbm_budget=10, max_batch=1, clock=clock, timeout_s=0.05)
    sch.register_stream(7, 1)
    sch.register_stream(8, 1)
    st = drive(sch, clock, [(0.0, 7, 0), (0.0, 8, 1)], horizon=0.06)
    assert st.failed == 1 and st.completed == 1 and st.timed_out == 1
    assert ex.slots == 63 and len(sch.quarantine) == 1    # withheld while its work may run
    drive(sch, clock, [], horizon=0.05)
    assert ex.slots == 64 and not sch.quarantine          # released once it ended
    assert st.failed == 1 and st.completed == 1


def test_batch_that_never_ends_stops_the_loop():
    clock = FakeClock()
    ex = FakeExecutor(clock, hang_streams={7})
    sch = Scheduler(ex, hbm_budget=10, max_batch=1, clock=clock, timeout_s=0.05)
    sch.register_stream(7, 1)
    with pytest.raises(ServingStalled):
        drive(sch, clock, [(0.0, 7, 0)], horizon=0.5)
    assert ex.slots == 63                                 # never handed to new frames


def test_unknown_device_error_stops_the_loop():
    class Lost(FakeExecutor):
        def done(self, h):
            raise RuntimeError("device lost")
    clock = FakeClock()
    sch = Scheduler(Lost(clock), hbm_budget=10, clock=clock)
    sch.register_stream(0, 1)
    with pytest.raises(RuntimeError, match="device lost"):
        drive(sch, clock, [(0.0, 0, 0)], horizon=0.05)


def test_stream_removal_drops_queued_frames_only():
    clock = FakeClock()
    ex = FakeExecutor(clock, delay=0.05)
    sch = Scheduler(ex, hbm_budget=10, max_batch=2, max_inflight=1, clock=clock)
    sch.register_stream(0, 1)
    sch.register_stream(1, 1)
    sch.t0 = clock()
    for k in range(6):
        sch.arrive(Frame(k % 2, k, 0.0))
    sch.launch()                                   # frames 0, 1 in flight
    sch.remove_stream(1)                           # drops queued frames 3, 5
    assert sch.stats.dropped_frames == 2
    # frame 1 of the removed stream is still in flight: its map stays resident
    # and its footprint stays counted until that batch ends
    assert 1 in ex.admitted and sch.used == 2 and ex.evicted == []
    sch.arrive(Frame(1, 99, 0.0))                  # arrives after removal: dropped
    assert sch.stats.dropped_frames == 3
    st = drive(sch, clock, [], horizon=0.5)
    assert st.completed == 4                       # 0, 1 (in flight) + 2, 4
    assert ex.evicted == [1] and 1 not in ex.admitted and sch.used == 1


@pytest.mark.parametrize("mode", ["batched", "per_frame"])
def test_summary_fields(mode):
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, hbm_budget=10, mode=mode, clock=clock)
    sch.register_stream(0, 1)
    st = drive(sch, clock, [(0.001 * k, 0, k) for k in range(10)], horizon=0.1)
    st.wall_s = 0.1
    s = st.summary()
    assert s["frames"] == 10 and s["p99_ms"] >= s["p50_ms"] > 0 and s["frames_per_s"] == 100.0

