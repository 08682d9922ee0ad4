"""Continuous-batching serving loop for many camera streams.

Frames from many streams arrive over time.  Each frame is one stereo pair
matched plus search by projection against its stream's local map (the map is
device-resident from admission on, Section IV-E's "transfer only what is
needed").  The scheduler

  * admits streams while their device footprint fits the HBM budget,
  * queues arriving frames (FIFO),
  * whenever an in-flight slot frees up, coalesces the pending frames into one
    batch (up to `max_batch`) and submits it, so work that arrives while other
    batches run is admitted as soon as capacity frees up; up to `max_inflight`
    batches run concurrently on separate HIP streams,
  * stamps each frame's latency from its arrival time to the moment the host
    sees its batch complete (frame upload included).

`mode="per_frame"` serves the same arrivals through the single-frame calls,
one frame at a time as it arrives (the plain per-frame GPU path), for the
comparison at equal p99 latency.

The scheduler only talks to an executor (`launch`, `done`, `release`, `admit`,
`evict`), so its logic is tested on the CPU with a fake executor.  `done(h)`
returns whether the batch's device work has ended; it raises `BatchFailed`
when the work ended with an error (the batch's slots may then be reused), and
any other exception means the device state is unknown, which stops the loop.
A batch that outlives `timeout_s` is reported failed at once, but its slots
stay withheld until the executor reports its work ended; if that does not
happen within another `timeout_s`, the loop stops with an error rather than
hand the slots to new frames.  A removed stream's map stays resident until
its last in-flight batch has ended.

Streams whose local map changes from frame to frame (Update Local Map's
output, Section II-D) are served sequentially, as tracking runs: with
`sequential=True` a batch takes, in FIFO order, at most one frame per stream
and no frame of a stream that still has a frame in flight, so the executor
can edit the stream's device map in place (ft_map_update, on the batch's HIP
stream, before the batch) with no batch reading it meanwhile.
"""
from __future__ import annotations

import collections
import ctypes as ct
import time
from dataclasses import dataclass, field

import numpy as np


class BatchFailed(RuntimeError):
    """A batch's device work ended with an error; its slots may be reused."""


class ServingStalled(RuntimeError):
    """A timed-out batch never reported completion: its slots cannot be
    handed to new frames, so serving stops."""


@dataclass
class Frame:
    stream: int
    seq: int
    arrival: float          # seconds since the start of the run
    done: float = -1.0
    failed: bool = False


@dataclass
class Stats:
    completed: int = 0
    failed: int = 0
    rejected_streams: list = field(default_factory=list)
    dropped_frames: int = 0
    batches: int = 0
    timed_out: int = 0
    max_overlap: int = 0         # largest number of batches in flight at once
    latencies_ms: list = field(default_factory=list)
    wall_s: float = 0.0

    def summary(self) -> dict:
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"frames": self.completed, "failed": self.failed,
                "dropped_frames": self.dropped_frames, "rejected_streams": self.rejected_streams,
                "batches": self.batches, "timed_out": self.timed_out, "max_overlap": self.max_overlap,
                "frames_per_s": self.completed / self.wall_s if self.wall_s > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_batch": self.completed / max(self.batches, 1)}


class Scheduler:
    """Stream registry, admission, FIFO coalescing and latency accounting."""

    def __init__(self, executor, hbm_budget: int, max_batch: int = 64, max_inflight: int = 4,
                 mode: str = "batched", clock=time.perf_counter, timeout_s: float = 10.0,
                 sequential: bool = False):
        assert mode in ("batched", "per_frame")
        self.sequential = sequential
        self.ex = executor
        self.budget = hbm_budget
        self.used = 0
        self.max_batch = max_batch if mode == "batched" else 1
        self.max_inflight = max_inflight
        self.mode = mode
        self.clock = clock
        self.timeout_s = timeout_s
        self.streams = {}
        self.pending = collections.deque()
        self.inflight = []           # (handle, frames, launch time)
        self.quarantine = []         # (handle, time-out time): failed, slots still withheld
        self.evicting = set()        # removed streams whose batches are still in flight
        self.stats = Stats()
        self.t0 = None

    # -- admission ---------------------------------------------------------
    def register_stream(self, sid: int, footprint: int) -> bool:
        if self.used + footprint > self.budget:
            self.stats.rejected_streams.append(sid)
            return False
        self.ex.admit(sid)
        self.streams[sid] = footprint
        self.used += footprint
        return True

    def remove_stream(self, sid: int):
        """Drop a stream: its queued frames are dropped, its in-flight frames
        finish (their results are simply not used).  Its map leaves the device,
        and its footprint the budget, once no batch in flight reads it."""
        if sid not in self.streams:
            return
        kept = collections.deque(f for f in self.pending if f.stream != sid)
        self.stats.dropped_frames += len(self.pending) - len(kept)
        self.pending = kept
        self.evicting.add(sid)
        self._finish_evictions()

    def _stream_busy(self, sid) -> bool:
        return any(f.stream == sid for _, frames, _ in self.inflight for f in frames) or \
            any(f.stream == sid for _, frames, _ in self.quarantine for f in frames)

    def _finish_evictions(self):
        for sid in [s for s in self.evicting if not self._stream_busy(s)]:
            self.evicting.discard(sid)
            self.used -= self.streams.pop(sid)
            self.ex.evict(sid)

    def arrive(self, frame: Frame):
        if frame.stream in self.streams and frame.stream not in self.evicting:
            self.pending.append(frame)
        else:
            self.stats.dropped_frames += 1

    # -- one scheduling step ------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    def _ended(self, h) -> tuple:
        """(work ended, ended with an error) for one batch."""
        try:
            return bool(self.ex.done(h)), False
        except BatchFailed:
            return True, True

    def poll(self):
        still = []
        for h, frames, t_launch in self.inflight:
            ended, err = self._ended(h)
            timed_out = not ended and self.now() - t_launch > self.timeout_s
            if ended or timed_out:
                t = self.now()
                for f in frames:
                    f.done = t
                    if err or timed_out:
                        f.failed = True
                        self.stats.failed += 1
                    else:
                        self.stats.completed += 1
                        self.stats.latencies_ms.append((t - f.arrival) * 1e3)
                if ended:
                    self.ex.release(h)
                else:
                    # reported failed, but its kernels may still write its
                    # slots: they stay withheld until the work has ended
                    self.stats.timed_out += 1
                    self.quarantine.append((h, frames, t))
            else:
                still.append((h, frames, t_launch))
        self.inflight = still
        held = []
        for h, frames, t_out in self.quarantine:
            if self._ended(h)[0]:
                self.ex.release(h)
            elif self.now() - t_out > self.timeout_s:
                raise ServingStalled(f"batch {h} has not ended {self.timeout_s} s after its time-out")
            else:
                held.append((h, frames, t_out))
        self.quarantine = held
        if self.evicting:
            self._finish_evictions()

    def launch(self) -> bool:
        if not self.pending or len(self.inflight) >= self.max_inflight:
            return False
        n = min(self.max_batch, len(self.pending), self.ex.free_slots())
        if n <= 0:
            return False
        if self.sequential:
            busy = {f.stream for _, fr, _ in self.inflight + self.quarantine for f in fr}
            frames, kept = [], collections.deque()
            for f in self.pending:
                if len(frames) < n and f.stream not in busy:
                    frames.append(f)
                    busy.add(f.stream)
                else:
                    kept.append(f)
            if not frames:
                return False
            self.pending = kept
        else:
            frames = [self.pending.popleft() for _ in range(n)]
        try:
            h = self.ex.launch(frames, per_frame=self.mode == "per_frame")
        except Exception:
            for f in frames:
                f.failed = True
                self.stats.failed += 1
            return True
        self.inflight.append((h, frames, self.now()))
        self.stats.batches += 1
        self.stats.max_overlap = max(self.stats.max_overlap, len(self.inflight))
        return True

    def run(self, arrivals) -> Stats:
        """Serve `arrivals` = [(time_s, stream, seq)] in real time."""
        self.t0 = self.clock()
        i, n = 0, len(arrivals)
        end = arrivals[-1][0] if n else 0.0
        while True:
            now = self.now()
            while i < n and arrivals[i][0] <= now:
                t, s, q = arrivals[i]
                self.arrive(Frame(s, q, t))
                i += 1
            self.poll()
            while self.launch():
                pass
            if i >= n and not self.pending and not self.inflight and not self.quarantine:
                break
        self.stats.wall_s = max(self.now(), end)
        return self.stats


# --------------------------------------------------------------------------
# Device executor
# --------------------------------------------------------------------------
def _carve(sizes):
    """Offsets of consecutive 256-byte aligned parts; returns (offsets, total)."""
    off, out = 0, {}
    for k, n in sizes:
        out[k] = off
        off += (n + 255) // 256 * 256
    return out, off


def _input_layout(n: int):
    """One frame's keypoint inputs for `n` keypoints per image, packed."""
    return _carve([("Lx", 4 * n), ("Ly", 4 * n), ("Rx", 4 * n), ("Ry", 4 * n),
                   ("Ldesc", 32 * n), ("Rdesc", 32 * n), ("Loct", n), ("Roct", n),
                   ("pre0", n), ("pre1", n)])


def _output_layout(kp: int, nm: int):
    return _carve([("right_idx", 4 * kp), ("dist", 4 * kp), ("u_right", 4 * kp), ("depth", 4 * kp),
                   ("sad", 4 * kp), ("xyz", 12 * kp), ("n_stereo", 4), ("mp_match", 8 * nm),
                   ("mp_dist", 8 * nm), ("kp_match", 8 * kp), ("n_search", 8)])


class DeviceExecutor:
    """Runs batches through the HIP library with stream maps resident on the
    device.

    Every in-flight frame slot owns one device region: the frame's packed
    inputs followed by its outputs.  Each pooled frame of an admitted stream
    is packed once into a pinned host arena (ft_host_alloc), as a frame
    producer would write it.  A launch uploads its frames with one gather
    copy (ft_upload) and submits job descriptors patched from per-frame
    templates: a template is built once per pooled frame for slot 0, and the
    words that hold slot addresses are shifted by the slot's offset.

    A stream with per-frame map edits ("edits", point ids) holds its map in
    device arrays of its map size; before a frame of sequence number k is
    launched, the edits of sequence numbers since the map's last frame up to
    k are applied in order on the batch's HIP stream by ft_map_update, which
    reads the inserted points from the stream's pinned host block (packed
    once at admission, as a local-map producer would write them): no copy
    command per edit.  Removals are given as point ids with the stream's id
    record (which point each slot holds), which the library translates and
    keeps; each edit's call arguments are prepared at admission."""

    def __init__(self, streams, max_batch: int = 64, max_inflight: int = 4, max_kp: int = 4096,
                 device: str = "cuda"):
        import torch

        from . import binding as ft
        self.torch, self.ft = torch, ft
        self.streams = {s["id"]: s for s in streams}
        self.max_batch, self.max_inflight = max_batch, max_inflight
        n_map = max(max(s["n_map"] for s in streams), 1)
        # streams with per-frame map edits: id record, prepared edits
        self.id_rec, self.id_struct, self.edit_structs, self.map_seq, self.map_struct = {}, {}, {}, {}, {}
        self.ins_block, self.ins_pts = {}, {}
        self.ctx = ft.Context(ft.default_limits(max_kp_per_image=max_kp, max_map_points=n_map,
                                                max_batch_frames=max_batch, max_inflight=max_inflight))
        self.hip_streams = [torch.cuda.Stream(device=device) for _ in range(max_inflight)]
        self.in_max = _input_layout(max_kp)[1]
        self.out_off, out_bytes = _output_layout(max_kp, n_map)
        self.slot_bytes = self.in_max + out_bytes
        n_slots = max_batch * max_inflight
        self.dev = torch.empty((n_slots, self.slot_bytes), dtype=torch.uint8, device=device)
        self.dev_base = self.dev.data_ptr()
        self.free = list(range(n_slots))
        self.outs = [self._out_views(k, max_kp, n_map) for k in range(n_slots)]
        # host arena: every pooled frame of every stream, packed
        self.arena_off = {}
        off = 0
        for s in streams:
            for q, f in enumerate(s["frames"]):
                self.arena_off[(s["id"], q)] = off
                off += _input_layout(len(f["left"]["x"]))[1]
        self.arena_bytes = max(off, 256)
        self.arena = self.ctx.ft_host_alloc(self.arena_bytes)
        self.arena_np = np.ctypeslib.as_array((ct.c_uint8 * self.arena_bytes).from_address(self.arena))
        self.maps = {}
        self.pyr = {}          # (stream, id(pyramid dict)) -> device tensor, per stream
        self.on_release = None # optional hook(handle) called before a batch's slots are freed
        self.tmpl = {}         # (stream, pool index) -> (template words, slot mask, packed bytes)
        self.packed = {}       # (stream, pool index) -> packed bytes in the arena
        self.device = device
        self.handles = {}
        self.next_h = 0

    def _out_views(self, slot, kp, nm):
        torch = self.torch
        row = self.dev[slot]

        def part(key, nbytes, dtype, shape):
            o = self.in_max + self.out_off[key]
            return row[o:o + nbytes].view(dtype).view(shape)
        i32, f32 = torch.int32, torch.float32
        return {"right_idx": part("right_idx", 4 * kp, i32, (kp,)), "dist": part("dist", 4 * kp, i32, (kp,)),
                "u_right": part("u_right", 4 * kp, f32, (kp,)), "depth": part("depth", 4 * kp, f32, (kp,)),
                "sad": part("sad", 4 * kp, i32, (kp,)), "xyz": part("xyz", 12 * kp, f32, (kp, 3)),
                "n_stereo": part("n_stereo", 4, i32, (1,)),
                "mp_match": part("mp_match", 8 * nm, i32, (2, nm)), "mp_dist": part("mp_dist", 8 * nm, i32, (2, nm)),
                "kp_match": part("kp_match", 8 * kp, i32, (2, kp)), "n_search": part("n_search", 8, i32, (2,))}

    # -- residency -----------------------------------------------------------
    def admit(self, sid):
        if sid in self.maps:
            return
        torch = self.torch
        s = self.streams[sid]
        if "edits" in s:
            ids0 = np.asarray(s["map_ids0"], dtype=np.int64)
            mp = {k: v[ids0] for k, v in s["points"].items()}
            rec = {"slot_id": np.zeros(len(ids0), dtype=np.int32),     # the map's capacity
                   "slot_of": np.full(len(s["points"]["dmin"]), -1, dtype=np.int32)}
            self.id_rec[sid] = rec
            self.id_struct[sid] = self.ft.ft_map_ids(rec["slot_id"].ctypes.data, rec["slot_of"].ctypes.data,
                                                     len(rec["slot_of"]))
            self._reset_record(sid)
            self._pack_inserts(sid)
        else:
            mp = s["frames"][0]["map"]
        self.maps[sid] = {k: torch.from_numpy(np.ascontiguousarray(v)).to(self.device) for k, v in mp.items()}
        m = self.maps[sid]
        self.map_struct[sid] = self.ft.ft_map_points(len(mp["dmin"]), m["pos"].data_ptr(), m["normal"].data_ptr(),
                                                     m["dmin"].data_ptr(), m["dmax"].data_ptr(),
                                                     m["desc"].data_ptr())
        if "edits" in s:   # every edit's call arguments, prepared once (arrays kept alive here)
            keep, structs = [], []
            for q, e in enumerate(s["edits"]):
                if e is None:
                    structs.append(None)
                    continue
                rem = np.ascontiguousarray(e["remove_ids"], dtype=np.int32)
                iid = np.ascontiguousarray(e["insert_ids"], dtype=np.int32)
                keep += [rem, iid]
                ins = self.ins_pts[sid][q]
                structs.append(self.ft.ft_map_edit(len(rem), rem.ctypes.data if len(rem) else None,
                                                   ins if ins is not None else self.ft.ft_map_points(),
                                                   iid.ctypes.data if len(iid) else None,
                                                   ct.pointer(self.id_struct[sid])))
            self.edit_structs[sid] = (structs, keep)
        for key, p in self._pyramids(sid).items():
            self.pyr[key] = torch.from_numpy(p["data"]).to(self.device)
        for q, f in enumerate(s["frames"]):
            if (sid, q) not in self.packed:   # packed once: an upload may still read it
                self.packed[(sid, q)] = self._pack(f, self.arena_off[(sid, q)])
            self.tmpl[(sid, q)] = self._template(sid, f) + (self.packed[(sid, q)],)

    def evict(self, sid):
        """Frees what the stream holds on the device (exactly what footprint
        counts); the scheduler calls it once no batch in flight reads it."""
        self.maps.pop(sid, None)
        for d in (self.id_rec, self.id_struct, self.edit_structs, self.map_seq, self.map_struct, self.ins_pts):
            d.pop(sid, None)
        if sid in self.ins_block:
            self.ctx.ft_host_free(self.ins_block.pop(sid))
        for k in [k for k in self.tmpl if k[0] == sid]:
            del self.tmpl[k]
        for k in [k for k in self.pyr if k[0] == sid]:
            del self.pyr[k]

    def _pyramids(self, sid) -> dict:
        """The distinct image pyramids of a stream's pooled frames."""
        out = {}
        for f in self.streams[sid]["frames"]:
            for key in ("pyr_left", "pyr_right"):
                if key in f:
                    out[(sid, id(f[key]))] = f[key]
        return out

    def footprint(self, sid) -> int:
        """Device bytes a stream holds while admitted: its map (64 bytes per
        point) and its own copy of each distinct pyramid of its pooled frames."""
        return self.streams[sid]["map_bytes"] + sum(p["data"].size for p in self._pyramids(sid).values())

    def resident_bytes(self) -> int:
        """Device bytes held for admitted streams (maps and pyramids)."""
        return (sum(t.numel() * t.element_size() for m in self.maps.values() for t in m.values()) +
                sum(t.numel() for t in self.pyr.values()))

    def _pack_inserts(self, sid):
        """Every edit's inserted points, packed into one pinned host block of
        the context (five 256-byte aligned arrays per edit)."""
        s = self.streams[sid]
        fields = (("pos", 12), ("normal", 12), ("dmin", 4), ("dmax", 4), ("desc", 32))
        sizes = [sum(-(-w * len(e["insert_ids"]) // 256) * 256 for _, w in fields) if e is not None else 0
                 for e in s["edits"]]
        total = max(sum(sizes), 256)
        base = self.ctx.ft_host_alloc(total)
        self.ins_block[sid] = base
        view = np.ctypeslib.as_array((ct.c_uint8 * total).from_address(base))
        pts, at = [], 0
        for e in s["edits"]:
            m = 0 if e is None else len(e["insert_ids"])
            if not m:
                pts.append(None)
                continue
            addr = {}
            for key, w in fields:
                b = np.ascontiguousarray(s["points"][key][e["insert_ids"]]).view(np.uint8).reshape(-1)
                view[at:at + b.size] = b
                addr[key] = base + at
                at += -(-w * m // 256) * 256
            pts.append(self.ft.ft_map_points(m, addr["pos"], addr["normal"], addr["dmin"], addr["dmax"],
                                             addr["desc"]))
        self.ins_pts[sid] = pts

    def _reset_record(self, sid):
        ids0 = np.asarray(self.streams[sid]["map_ids0"], dtype=np.int64)
        rec = self.id_rec[sid]
        rec["slot_id"][:len(ids0)] = ids0
        rec["slot_of"][:] = -1
        rec["slot_of"][ids0] = np.arange(len(ids0))
        self.map_seq[sid] = 0

    def reset_map(self, sid):
        """Upload a stream's first map again (a new run's sequence numbers
        start at 0); the device is synchronised first."""
        s = self.streams[sid]
        self.torch.cuda.synchronize()
        ids0 = np.asarray(s["map_ids0"], dtype=np.int64)
        for k, t in self.maps[sid].items():
            t[:len(ids0)].copy_(self.torch.from_numpy(np.ascontiguousarray(s["points"][k][ids0])))
        self._reset_record(sid)
        self.map_struct[sid].n = len(ids0)

    def _edit_maps(self, frames, hs):
        """Bring each edited stream's device map from its last frame's map to
        its frame's, on HIP stream `hs`: round r applies every stream's r-th
        pending edit in one ft_map_update_many call (a stream is normally one
        edit behind)."""
        pending = []
        for fr in frames:
            sid = fr.stream
            if sid in self.map_seq:
                assert fr.seq >= self.map_seq[sid], "frames of an edited map arrive in order"
                if fr.seq > self.map_seq[sid]:
                    pending.append((sid, self.map_seq[sid] + 1, fr.seq))
                    self.map_seq[sid] = fr.seq
        while pending:
            maps, caps, edits, rest = [], [], [], []
            for sid, k, last in pending:
                s = self.streams[sid]
                maps.append(self.map_struct[sid])
                caps.append(self.maps[sid]["dmin"].numel())
                edits.append(self.edit_structs[sid][0][k % len(s["frames"])])
                if k < last:
                    rest.append((sid, k + 1, last))
            self.ctx.ft_map_update_many(maps, caps, edits, stream=hs)
            pending = rest

    def _pack(self, f, at):
        L, R = f["left"], f["right"]
        n = len(L["x"])
        lay, total = _input_layout(n)
        a = self.arena_np[at:at + total]
        a[:] = 0

        def put(key, arr):
            b = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
            a[lay[key]:lay[key] + b.size] = b
        put("Lx", L["x"].astype(np.float32)); put("Ly", L["y"].astype(np.float32))
        put("Rx", R["x"].astype(np.float32)); put("Ry", R["y"].astype(np.float32))
        put("Ldesc", L["desc"]); put("Rdesc", R["desc"])
        put("Loct", L["octave"]); put("Roct", R["octave"])
        for v, spec in enumerate(f["search"]):
            put("pre%d" % v, spec["preassigned"].astype(np.uint8))
        return total

    # -- jobs ------------------------------------------------------------------
    def _template(self, sid, f):
        """Job words for slot 0 and the mask of words holding slot addresses
        (found by building the job for slots 0 and 1 and comparing)."""
        w0 = np.frombuffer(bytes(self._job(sid, f, 0)), dtype=np.uint64)
        w1 = np.frombuffer(bytes(self._job(sid, f, 1)), dtype=np.uint64)
        mask = (w0 != w1).astype(np.uint64)
        assert np.all((w1 - w0)[mask == 1] == np.uint64(self.slot_bytes)), "job words move with the slot"
        return w0.copy(), mask

    def _job(self, sid, f, slot):
        ft = self.ft
        n = len(f["left"]["x"])
        base = self.dev_base + slot * self.slot_bytes
        lay = _input_layout(n)[0]
        o = self.outs[slot]
        sc = f["scales"]
        j = ft.ft_frame_job()
        j.left = ft.ft_keypoints(n, base + lay["Lx"], base + lay["Ly"], base + lay["Loct"], base + lay["Ldesc"])
        j.right = ft.ft_keypoints(n, base + lay["Rx"], base + lay["Ry"], base + lay["Roct"], base + lay["Rdesc"])
        j.scales = ft._scales(sc)
        if f["kind"] == "pinhole":
            j.kind = ft.FT_JOB_PINHOLE
            for key, dst in (("pyr_left", "pyr_left"), ("pyr_right", "pyr_right")):
                p = f[key]
                s = ft.ft_pyramid()
                s.data = self.pyr[(sid, id(p))].data_ptr()
                s.offset[:] = [int(v) for v in p["offset"]]
                s.width[:] = [int(v) for v in p["width"]]
                s.height[:] = [int(v) for v in p["height"]]
                setattr(j, dst, s)
            c, sp = f["stereo_cam"], f["stereo_params"]
            j.pinhole = ft.ft_pinhole_stereo(float(c["fx"]), float(c["bf"]), float(c["b"]), int(c["rows"]))
            j.pinhole_params = ft.ft_pinhole_params(sp["th_orb"], sp["half_win"], sp["half_range"],
                                                    sp["level_window"], sp["median_num"], sp["median_den"],
                                                    sp["band"])
            j.pinhole_out = ft.ft_pinhole_out(o["right_idx"].data_ptr(), o["dist"].data_ptr(),
                                              o["u_right"].data_ptr(), o["depth"].data_ptr(),
                                              o["sad"].data_ptr(), o["n_stereo"].data_ptr())
            j.use_u_right = 1
        else:
            j.kind = ft.FT_JOB_FISHEYE
            c, sp = f["stereo_cam"], f["stereo_params"]
            fs = ft.ft_fisheye_stereo()
            fs.left, fs.right = ft._kb(c["left"]), ft._kb(c["right"])
            fs.R_lr[:] = [float(v) for v in np.asarray(c["R_lr"], np.float32).reshape(-1)]
            fs.t_lr[:] = [float(v) for v in c["t_lr"]]
            fs.overlap_left[:] = [float(v) for v in c["overlap_left"]]
            fs.overlap_right[:] = [float(v) for v in c["overlap_right"]]
            j.fisheye = fs
            j.fisheye_params = ft.ft_fisheye_params(sp["ratio_num"], sp["ratio_den"], sp["newton_iters"], 0,
                                                    sp["cos_parallax_max"], sp["chi2"],
                                                    float(np.deg2rad(sp["max_theta_deg"])), sp["newton_tol"])
            j.fisheye_out = ft.ft_fisheye_out(o["right_idx"].data_ptr(), o["dist"].data_ptr(),
                                              o["depth"].data_ptr(), o["xyz"].data_ptr(),
                                              o["n_stereo"].data_ptr())
        j.map = ft.ft_map_points.from_buffer_copy(bytes(self.map_struct[sid]))
        j.search_params = ft.search_params_struct(f["search_params"])
        j.n_views = len(f["search"])
        for v, spec in enumerate(f["search"]):
            j.cam[v] = ft.search_camera_struct(spec["cam"])
            j.grid[v] = ft.ft_grid(*spec["grid"])
            j.preassigned[v] = base + lay["pre%d" % v]
            j.search_out[v] = ft.ft_search_out(o["mp_match"][v].data_ptr(), o["mp_dist"][v].data_ptr(),
                                               o["kp_match"][v].data_ptr(), o["n_search"][v:v + 1].data_ptr())
        return j

    def autotune(self, n: int | None = None, cache_path: str | None = None):
        """Pick launch shapes on a batch of up to `n` pooled frames of the
        admitted streams (uploaded to slots 0.., then timed by ft_autotune)."""
        ft = self.ft
        n = min(n or self.max_batch, self.max_batch)
        keys = [k for k in self.tmpl][:n]
        if not keys:
            return None
        jobs = np.stack([self.tmpl[k][0] + self.tmpl[k][1] * np.uint64(i * self.slot_bytes)
                         for i, k in enumerate(keys)])
        segs = np.array([(self.arena + self.arena_off[k], self.dev_base + i * self.slot_bytes, self.tmpl[k][2])
                         for i, k in enumerate(keys)], dtype=np.int64)
        hs = self.hip_streams[0]
        self.ctx.ft_upload(segs, hs)
        structs = [ft.ft_frame_job.from_buffer_copy(row.tobytes()) for row in jobs]
        return self.ctx.ft_autotune(structs, cache_path=cache_path, stream=hs)

    # -- executor protocol -----------------------------------------------------
    def free_slots(self) -> int:
        return len(self.free)

    def launch(self, frames, per_frame=False):
        # single-frame calls share the context's one workspace: keep them on one
        # stream; each in-flight batch owns its own workspace lane
        lane = 0 if per_frame else self.next_h % self.max_inflight
        hs = self.hip_streams[lane]
        n = len(frames)
        if self.map_seq:
            self._edit_maps(frames, hs)
        slots = [self.free.pop() for _ in range(n)]
        keys = [(fr.stream, fr.seq % len(self.streams[fr.stream]["frames"])) for fr in frames]
        t = [self.tmpl[k] for k in keys]
        shift = np.array(slots, dtype=np.uint64) * np.uint64(self.slot_bytes)
        jobs = np.stack([w for w, _, _ in t]) + np.stack([m for _, m, _ in t]) * shift[:, None]
        if self.map_seq:
            n_word = jobs.view(np.int32)
            at = self.ft.ft_frame_job.map.offset // 4    # ft_map_points.n: the map's current size
            for i, fr in enumerate(frames):
                if fr.stream in self.map_struct and fr.stream in self.map_seq:
                    n_word[i, at] = self.map_struct[fr.stream].n
        segs = np.empty((n, 3), dtype=np.int64)
        segs[:, 0] = [self.arena + self.arena_off[k] for k in keys]
        segs[:, 1] = self.dev_base + np.array(slots, dtype=np.int64) * self.slot_bytes
        segs[:, 2] = [b for _, _, b in t]
        self.ctx.ft_upload(segs, hs)
        if per_frame:
            self._run_single(self.ft.ft_frame_job.from_buffer_copy(jobs[0].tobytes()), hs)
            ev = self.torch.cuda.Event()
            ev.record(hs)
            token = ("event", ev)
        else:
            token = ("ticket", self.ctx.ft_batch_submit_raw(jobs.ctypes.data, n, hs))
        h = self.next_h
        self.next_h += 1
        self.handles[h] = (token, slots, frames)
        return h

    def _run_single(self, j, hs):
        ctx, ft = self.ctx, self.ft
        if j.kind == ft.FT_JOB_PINHOLE:
            ctx.ft_stereo_match_pinhole(j.left, j.right, j.pyr_left, j.pyr_right, j.scales, j.pinhole,
                                        j.pinhole_params, j.pinhole_out, stream=hs)
        else:
            ctx.ft_stereo_match_fisheye(j.left, j.right, j.scales, j.fisheye, j.fisheye_params,
                                        j.fisheye_out, stream=hs)
        for v in range(j.n_views):
            kps = j.left if v == 0 else j.right
            ur = j.pinhole_out.u_right if (v == 0 and j.kind == ft.FT_JOB_PINHOLE and j.use_u_right) else None
            ctx.ft_search_local_points(j.map, j.cam[v], kps, ur, j.preassigned[v], j.grid[v], j.scales,
                                       j.search_params, j.search_out[v], stream=hs)

    def done(self, h) -> bool:
        token = self.handles[h][0]
        if token[0] == "event":
            return token[1].query()
        return self.ctx.ft_batch_poll(token[1])

    def release(self, h):
        if self.on_release is not None:
            self.on_release(h)
        _, slots, _ = self.handles.pop(h)
        self.free.extend(slots)

    def results(self, slot: int, kind: str, n: int, n_map: int, n_views: int, sync: bool = True) -> dict:
        """Copy one slot's outputs to the host (synchronises the device unless
        `sync` is false, for a slot whose batch is known to have ended)."""
        o = self.outs[slot]
        if sync:
            self.torch.cuda.synchronize()
        st = {"right_idx": o["right_idx"][:n].cpu().numpy(), "dist": o["dist"][:n].cpu().numpy(),
              "n_matches": int(o["n_stereo"][0])}
        if kind == "pinhole":
            st.update(u_right=o["u_right"][:n].cpu().numpy(), depth=o["depth"][:n].cpu().numpy(),
                      sad=o["sad"][:n].cpu().numpy())
        else:
            st.update(depth=o["depth"][:n].cpu().numpy(), xyz=o["xyz"][:n].cpu().numpy())
        search = [{"mp_match": o["mp_match"][v][:n_map].cpu().numpy(),
                   "mp_dist": o["mp_dist"][v][:n_map].cpu().numpy(),
                   "kp_match": o["kp_match"][v][:n].cpu().numpy(),
                   "n_matches": int(o["n_search"][v])} for v in range(n_views)]
        return {"kind": kind, "stereo": st, "search": search}


def serve(streams, duration_s: float, speedup: float = 1.0, mode: str = "batched",
          max_batch: int = 64, max_inflight: int = 4, hbm_budget: int = 8 << 30, seed: int = 0,
          executor=None) -> dict:
    """Serve Poisson arrivals of every stream for `duration_s` seconds."""
    from synth.serving import poisson_arrivals
    ex = executor or DeviceExecutor(streams, max_batch=max_batch, max_inflight=max_inflight)
    sch = Scheduler(ex, hbm_budget, max_batch=max_batch, max_inflight=max_inflight, mode=mode,
                    sequential=any("edits" in s for s in streams))
    for s in streams:
        if sch.register_stream(s["id"], ex.footprint(s["id"])) and s["id"] in getattr(ex, "map_seq", {}):
            ex.reset_map(s["id"])
    arr = poisson_arrivals(np.random.default_rng(seed), streams, duration_s, speedup)
    arr = [a for a in arr if a[1] in sch.streams] + [a for a in arr if a[1] not in sch.streams]
    arr.sort()
    st = sch.run(arr)
    out = st.summary()
    out.update(mode=mode, speedup=speedup, offered_fps=len(arr) / duration_s, streams=len(streams))
    return out
