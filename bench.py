"""Benchmark: frame-pairs/s of stereo matching + local-map search on one MI355X.

One step = one batch submission of the 64-frame mixed workload (32 rectified
pinhole 752x480 frames and 32 fisheye 512x512 frames in seeded order,
300-3000 keypoints per image, 1k-20k local map points): for every frame,
stereo matching and search by projection in each camera view.  Inputs are
resident in device memory before the timed region.  Prints one JSON line.

Beside the headline the default run also reports:
  * latency of one 64-frame submission, and the same frames through the
    single-frame calls (the plain per-frame GPU path);
  * per-phase kernel times (HIP events) and the dominant kernel's roofline
    fraction, warm and cold (the 256 MB last-level cache flushed by a 512 MB
    write before every submission);
  * per-frame p50/p99 latency of the three single-frame workloads (pinhole
    1200 keypoints / 3000 map points, fisheye 1500 / 5000, clustered 3000 /
    20000);
  * the clustered scene over 64 seeds in one submission, with the search
    kernel's roofline on it;
  * the same 64 frames with every pinhole job building its two image
    pyramids on the device first (throughput, and the pyramid kernel's
    roofline warm and cold);
  * the last-frame search by projection (Initial Pose Estimation) on the
    pinhole frame and both fisheye views: per-call p50/p99;
  * ORB extraction of the benchmark's 64 pinhole images (FAST-9 corners on
    all eight levels, every corner described): images/s, corners per image,
    detection and description times and the detection kernel's roofline;
  * local-map maintenance on the device: a 20000-point map with 5% of its
    points replaced per edit, against uploading the whole map again;
  * a bounded serving sweep (32 camera streams, resident maps of 2k-40k
    points): per-frame path and continuous batching over the same Poisson
    arrivals, frames/s at equal p99, and a sample of frames served inside
    overlapping batches checked bit for bit against the same frames alone;
    then the same streams with 5% of every local map replaced before each
    frame (maps edited in place on the device, frames of a stream in order);
  * the CPU oracle on the same frames, one thread and on all host cores (the
    host's CPU model and core count recorded), and on each single-frame
    workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "frame-pairs/s (stereo + local-map search) on 1 MI355X; p50/p99 frame latency"
WORKLOAD = ("batched: 64 stereo frames, 32 pinhole 752x480 + 32 fisheye 512x512 (seeded order), "
            "300-3000 keypoints/image, 1k-20k local map points/frame, one submission per step")
FLUSH_BYTES = 512 << 20     # twice the MI355X last-level cache


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_search_bytes(frames):
    """Compulsory bytes of the search-by-projection kernel for one step.

    Per map point and view: 64 B record (position 12, normal 12, dmin 4, dmax 4,
    descriptor 32) read + 8 B (match, distance) written; per keypoint and view:
    x 4 + y 4 + level 1 + descriptor 32 + grid entry 4 read, + preassigned flag
    1 and right coordinate 4 where given.
    """
    total = 0
    for f in frames:
        nM = len(f["map"]["dmin"])
        for spec in f["search"]:
            nK = len(f[spec["image"]]["x"])
            per_kp = 45 + (1 if spec.get("preassigned") is not None else 0) + (4 if spec.get("use_u_right") else 0)
            total += nM * (64 + 8) + nK * per_kp
    return total


KERNEL_SOURCE = os.path.join(ROOT, "paper_2509_10757_amd", "csrc", "ft_kernels.hip")
ORB_SOURCE = os.path.join(ROOT, "paper_2509_10757_amd", "csrc", "ft_orb.hip")


def measured_traffic(kernel_key, workload, source=KERNEL_SOURCE):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what
    the counter reads for a plain copy of known size), or None when there is no
    summary for it on this workload or the kernel source changed since the
    counters were taken."""
    import glob
    import re
    digest = hashlib.sha256(open(source, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*pmc*.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if (rec.get("kernel_key") != kernel_key or rec.get("source_sha256") != digest or
                rec.get("workload", "mixed_batch64") != workload):
            continue
        return round(rec["fetch_kib"] * rec["fetch_scale"] * 1024 + rec["write_kib"] * rec["write_scale"] * 1024)
    return None


# ------------------------------------------------------------ CPU oracle ----
def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def _digest(res):
    h = hashlib.sha256()
    if "stereo" in res:
        for k in ("right_idx", "dist"):
            h.update(res["stereo"][k].tobytes())
    for s in res["search"]:
        for k in ("mp_match", "mp_dist", "kp_match"):
            h.update(s[k].tobytes())
    return h.hexdigest()[:16]


_POOL_FRAMES = None


def _oracle_worker(args):
    """Runs the oracle on frames w, w + P, w + 2P, ... (wrapping) for `budget`
    seconds; returns (frames done, digests of the first pass)."""
    w, P, budget = args
    import oracle
    frames = _POOL_FRAMES
    done, seen = 0, {}
    t0 = time.perf_counter()
    i = w
    while time.perf_counter() - t0 < budget:
        idx = i % len(frames)
        r = oracle.run_frame(frames[idx])
        if idx not in seen:
            seen[idx] = _digest(r)
        done += 1
        i += P
    return done, seen, time.perf_counter() - t0


def cpu_baseline(frames, single, budget_s=10.0, workers=None):
    """The oracle as it stands on the same frames: (i) one thread, in order;
    (ii) one process per host core (at most 16, the host share of one GPU),
    each taking every P-th frame.  Both runs hash their results; frames done
    by both must hash the same.  Also the oracle's time on each single-frame
    workload in `single` (name -> frame)."""
    import multiprocessing as mp

    import oracle
    global _POOL_FRAMES
    oracle._load()
    per_config = {}
    for name, f in single.items():
        o0 = time.perf_counter()
        oracle.run_frame(f)
        per_config[name] = round((time.perf_counter() - o0) * 1e3, 2)
    done, seen = 0, {}
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        idx = done % len(frames)
        r = oracle.run_frame(frames[idx])
        if idx not in seen:
            seen[idx] = _digest(r)
        done += 1
    dt1 = time.perf_counter() - t0
    single_run = {"value": round(done / dt1, 3), "unit": "frame-pairs/s", "cores": 1,
                  "sample": f"{done} frames of the 64-frame workload in order, {dt1:.1f} s"}
    info = host_info()
    P = workers or max(1, min(16, info["nproc"]))
    _POOL_FRAMES = frames
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        outs = pool.map(_oracle_worker, [(w, P, budget_s) for w in range(P)])
    dt = time.perf_counter() - t0
    _POOL_FRAMES = None
    total = sum(o[0] for o in outs)
    par_seen = {}
    for o in outs:
        par_seen.update(o[1])
    common = set(seen) & set(par_seen)
    identical = all(seen[k] == par_seen[k] for k in common)
    return {"value": round(total / dt, 3), "unit": "frame-pairs/s", "cores": P, "kind": "oracle",
            "sample": (f"{total} frames of the same 64-frame workload, {P} worker processes each taking "
                       f"every {P}-th frame (wrapping) for {budget_s:.0f} s; plain C oracle, unchanged"),
            "single_thread": single_run, "host": info, "single_frame_workloads_ms": per_config,
            "results_identical_to_single_thread": identical, "frames_compared": len(common)}


# -------------------------------------------------------------- serving ----
def same_results(a, b) -> bool:
    """Two device result dicts hold identical bits."""
    import numpy as np
    if ("stereo" in a) != ("stereo" in b) or len(a["search"]) != len(b["search"]):
        return False
    pairs = [(a["stereo"], b["stereo"])] if "stereo" in a else []
    pairs += list(zip(a["search"], b["search"]))
    for x, y in pairs:
        for k, v in x.items():
            if isinstance(v, np.ndarray):
                if not np.array_equal(v.view(np.uint8), y[k].view(np.uint8)):
                    return False
            elif v != y[k]:
                return False
    return True


def serving_sweep(duration_s, per_frame_rates, batched_rates, check_frames=24):
    """Serving 32 camera streams (20-30 Hz, resident maps of 2k-40k points):
    the per-frame path and continuous batching over the same Poisson arrivals,
    compressed in time by the given factors (ascending).  Each mode stops after
    the first rate it cannot keep up with (served < 90 % of offered).  Then a
    batched run whose first `check_frames` served frames are copied as their
    batches end (while other batches are in flight) and compared bit for bit
    with the same frames served alone through the single-frame calls."""
    import numpy as np

    from paper_2509_10757_amd import serve
    from synth.serving import make_streams
    log("generating the 32-stream serving workload")
    streams = make_streams()
    ex = serve.DeviceExecutor(streams, max_batch=64, max_inflight=4)
    for s in streams:
        ex.admit(s["id"])
    log("serving shapes", ex.autotune())
    rows, bound, knee, best = _sweep_modes(serve, ex, streams, duration_s, per_frame_rates, batched_rates)

    # served results (copied before the slots are reused) against the same
    # frames served alone
    captured = []

    def keep(h):
        if len(captured) >= check_frames:
            return
        _, slots, frames = ex.handles[h]
        for slot, fr in zip(slots, frames):
            s = ex.streams[fr.stream]
            q = fr.seq % len(s["frames"])
            f = s["frames"][q]
            captured.append((fr, f, ex.results(slot, f["kind"], len(f["left"]["x"]), len(f["map"]["dmin"]),
                                               len(f["search"]), sync=False)))
    ex.on_release = keep
    try:
        serve.serve(streams, min(duration_s, 0.3), speedup=batched_rates[len(batched_rates) // 2],
                    mode="batched", executor=ex)
    finally:
        ex.on_release = None
    bad = 0
    for fr, f, got in captured[:check_frames]:
        h = ex.launch([serve.Frame(fr.stream, fr.seq, 0.0)], per_frame=True)
        while not ex.done(h):
            pass
        alone = ex.results(ex.handles[h][1][0], f["kind"], len(f["left"]["x"]), len(f["map"]["dmin"]),
                           len(f["search"]), sync=False)
        ex.release(h)
        bad += not same_results(got, alone)
    out = {"streams": len(streams), "duration_s": duration_s, "runs": rows,
           **_at_bound(bound, knee, best),
           "served_frames_checked_against_alone": min(len(captured), check_frames),
           "served_frames_mismatching": bad}
    del ex

    # the same streams with 5 % of every local map replaced before each frame
    # (maps edited in place on the device, frames of a stream served in order)
    log("generating the 32-stream serving workload with 5% map churn per frame")
    cstreams = make_streams(map_churn=0.05)
    cex = serve.DeviceExecutor(cstreams, max_batch=64, max_inflight=4)
    for s in cstreams:
        cex.admit(s["id"])
    cex.autotune()
    crows, cbound, cknee, cbest = _sweep_modes(serve, cex, cstreams, duration_s, per_frame_rates,
                                               [4, 8, 16, 32, 48, 64, 96, 128, 192])
    out["map_churn"] = {"fraction_per_frame": 0.05, "runs": crows, **_at_bound(cbound, cknee, cbest),
                        "points_replaced_per_frame_mean": round(float(np.mean([len(s["edits"][1]["remove_ids"])
                                                                               for s in cstreams])), 1)}
    return out


def _sweep_modes(serve, ex, streams, duration_s, per_frame_rates, batched_rates):
    """Per-frame and batched runs over rising rates; each mode stops after the
    first rate it cannot keep up with.  Returns (rows, p99 bound, per-frame
    knee row, best batched row within the bound)."""
    rows = []
    for mode, rates in (("per_frame", per_frame_rates), ("batched", batched_rates)):
        for a in rates:
            r = serve.serve(streams, duration_s, speedup=a, mode=mode, executor=ex)
            log(mode, a, {k: round(v, 3) if isinstance(v, float) else v for k, v in r.items()
                          if k in ("frames_per_s", "p50_ms", "p99_ms", "offered_fps", "mean_batch", "max_overlap")})
            rows.append({k: r[k] for k in ("mode", "speedup", "offered_fps", "frames_per_s",
                                           "p50_ms", "p99_ms", "mean_batch", "max_overlap", "failed")})
            if r["frames_per_s"] < 0.9 * r["offered_fps"]:
                break
    pf = [r for r in rows if r["mode"] == "per_frame" and r["frames_per_s"] >= 0.95 * r["offered_fps"]]
    knee = max(pf, key=lambda r: r["offered_fps"]) if pf else min(
        (r for r in rows if r["mode"] == "per_frame"), key=lambda r: r["offered_fps"])
    bound = knee["p99_ms"]
    ok = [r for r in rows if r["mode"] == "batched" and r["p99_ms"] <= bound]
    best = max(ok, key=lambda r: r["frames_per_s"]) if ok else None
    return rows, bound, knee, best


def _at_bound(bound, knee, best):
    return {"p99_bound_ms": round(bound, 3), "per_frame_fps_at_bound": round(knee["frames_per_s"], 1),
            "batched_fps_at_bound": round(best["frames_per_s"], 1) if best else None,
            "batched_over_per_frame_at_equal_p99": (round(best["frames_per_s"] / knee["frames_per_s"], 2)
                                                    if best and knee["frames_per_s"] > 0 else None)}


# --------------------------------------------------------------- helpers ----
def percentiles(xs):
    import numpy as np
    a = np.asarray(xs)
    return {"p50": round(float(np.percentile(a, 50)), 4), "p99": round(float(np.percentile(a, 99)), 4)}


def phase_times(ctx, ft, submit, n, flush=None):
    """Average HIP-event time of each phase kernel over `n` eager submissions
    on one stream (each kernel runs alone); `flush()` runs before each."""
    ctx.ft_set_exec_mode(ft.FT_EXEC_EAGER)
    ctx.ft_context_enable_timing(True)
    for _ in range(n):
        if flush is not None:
            flush()
        submit()
    tm = ctx.ft_context_read_timing()
    ctx.ft_context_enable_timing(False)
    return {k: {"avg_us": round(ms / c * 1e3, 3), "launches": c} for k, (ms, c) in tm.items() if c}


def search_roofline(nbytes, us, traffic, note):
    achieved = nbytes / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "k_search_deal (search by projection)", "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic, "algorithmic_bytes_per_launch": nbytes, "avg_launch_us": round(us, 3),
            "timed": note}


def orb_leg(ctx, ft, frames, streams, steps, timing=True, flush=None):
    """ORB extraction of the benchmark's pinhole images (both images of each
    pinhole frame, 752x480, eight levels): detection (one kernel) then
    description of every detected corner, per image, images spread over the
    submission streams; throughput, corners per image, and HIP-event times of
    the detection and the description on one stream."""
    import numpy as np
    import torch

    import synth
    pat = synth.orb_pattern()
    sc = ft._scales(synth.scale_tables())
    imgs = [f[side] for f in frames if f["kind"] == "pinhole" for side in ("pyr_left", "pyr_right")]
    orbs = [ft.DeviceOrb(p, capacity=65536) for p in imgs]

    def run_all():
        for k, d in enumerate(orbs):
            st = streams[k % len(streams)]
            d.detect(ctx, sc, stream=st)
            d.describe(ctx, pat, stream=st)

    for _ in range(3):
        run_all()
    torch.cuda.synchronize()
    n = max(10, steps // 4)
    t0 = time.perf_counter()
    for _ in range(n):
        run_all()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    counts = [int(d.t["count"][0]) for d in orbs]
    out = {"workload": f"{len(imgs)} EuRoC-like 752x480 images (both images of the benchmark's pinhole frames), "
                       "8-level pyramids resident on the device; FAST threshold 20, every corner described",
           "images_per_s": round(len(imgs) * n / dt, 1), "rounds": n, "streams": len(streams),
           "corners_per_image": {"mean": round(float(np.mean(counts)), 1), "min": int(min(counts)),
                                 "max": int(max(counts))}}
    if not timing:
        return out

    def per_image(flush_each):
        st = streams[0]
        if flush_each is None:
            # The 64 detections back to back on one stream between two events,
            # then the 64 descriptions: average launch durations.  A description
            # is queued first, so the start event is taken when the GPU reaches
            # it, not while the host is still issuing the launches.
            n = len(orbs)
            orbs[0].describe(ctx, pat, stream=st)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(st)
            for d in orbs:
                d.detect(ctx, sc, stream=st)
            e[1].record(st)
            for d in orbs:
                d.describe(ctx, pat, stream=st)
            e[2].record(st)
            st.synchronize()
            return e[0].elapsed_time(e[1]) * 1e3 / n, e[1].elapsed_time(e[2]) * 1e3 / n
        # cold: each image behind a write of the last-level cache's size, its
        # detection and description bracketed by events
        evs = []
        for d in orbs:
            with torch.cuda.stream(st):
                flush_each()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(st)
            d.detect(ctx, sc, stream=st)
            e[1].record(st)
            d.describe(ctx, pat, stream=st)
            e[2].record(st)
            evs.append(e)
        st.synchronize()
        return (float(np.mean([e[0].elapsed_time(e[1]) * 1e3 for e in evs])),
                float(np.mean([e[1].elapsed_time(e[2]) * 1e3 for e in evs])))
    det_us, des_us = per_image(None)
    cold = per_image(flush)
    pyr_bytes = int(np.mean([d.pyr_t.numel() for d in orbs]))
    # detection: the pyramid read once, the smoothed pyramid written once, 14 B per corner written
    det_bytes = 2 * pyr_bytes + 14 * int(np.mean(counts))
    achieved = det_bytes / (det_us * 1e-6) / 1e9
    out["detect_us"] = round(det_us, 2)
    out["describe_us"] = round(des_us, 2)
    out["describe_ns_per_corner"] = round(des_us * 1e3 / max(np.mean(counts), 1), 2)
    out["cold"] = {"detect_us": round(cold[0], 2), "describe_us": round(cold[1], 2)}
    out["roofline"] = {"bound": "hbm", "kernel": "k_orb_detect (one image)", "achieved": round(achieved, 2),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                       "traffic": measured_traffic("k_orb_detect", "orb_images64", ORB_SOURCE),
                       "algorithmic_bytes_per_launch": det_bytes, "avg_launch_us": round(det_us, 3),
                       "timed": "HIP events around 64 detections queued back to back on one stream, "
                                "average per launch, warm caches"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of each oracle leg")
    ap.add_argument("--shapes", type=str, default="",
                    help="best_lanes,search_lanes[,aux_block] instead of autotuning")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel event passes")
    ap.add_argument("--exec", choices=["auto", "graph", "eager"], default="auto",
                    help="batch execution mode; auto times graph mode on 1-4 submission streams briefly")
    ap.add_argument("--streams", type=int, default=1, choices=[1, 2, 3, 4],
                    help="submission streams (with an explicit --exec)")
    ap.add_argument("--serving", type=float, default=0.6, metavar="SECONDS",
                    help="seconds per arrival rate of the serving sweep (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the single-frame workloads and the clustered batch")
    ap.add_argument("--only", choices=["mixed", "clustered", "pyramids", "orb", "fisheye", "pinhole"], default=None,
                    help="profiling runs: only the timed region of one workload, no other legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: the hot path is a single-GPU "
                                   "kernel set; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np

    import synth

    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 5}))
        return

    profiling = args.only is not None
    if args.only == "clustered":
        log("generating the clustered scene over 64 seeds")
        frames = synth.clustered_batch()
    else:
        log("generating the 64-frame workload")
        frames = synth.mixed_batch()
        if args.only in ("fisheye", "pinhole"):   # one kind's 32 frames of it (counter runs)
            frames = [f for f in frames if f["kind"] == args.only]
    n_frames = len(frames)

    single = {} if args.no_extra or profiling else {name: synth.workload(name)[0]
                                                   for name in sorted(synth.SINGLE_FRAME)}
    # CPU baselines first: the worker processes fork before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline and not profiling:
        log("cpu baseline")
        cpu = cpu_baseline(frames, single, budget_s=args.cpu_budget)
        log("cpu", cpu["value"], "frame-pairs/s on", cpu["cores"], "processes; one thread",
            cpu["single_thread"]["value"])

    import torch

    from paper_2509_10757_amd import binding as ft

    assert torch.cuda.is_available(), "bench needs a GPU"
    max_streams = 4
    ctx = ft.Context(ft.default_limits(max_batch_frames=n_frames, max_map_points=32768, max_inflight=8))
    # one private copy of the frames (inputs, workspace-independent outputs)
    # per submission stream, so batches in flight on different streams never
    # share a buffer
    build_pyr = args.only == "pyramids"   # profiling: the pinhole jobs build their pyramids first
    copies = [[ft.DeviceFrame(f, "cuda", build_pyramids=build_pyr) for f in frames]
              for _ in range(1 if profiling else max_streams)]
    dfs = copies[0]
    job_sets = [[d.job() for d in c] for c in copies]
    if args.only == "orb":
        r = orb_leg(ctx, ft, frames, [torch.cuda.current_stream()], args.steps, timing=False)
        print(json.dumps({"workload": "orb", **r}))
        return
    jobs = job_sets[0]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(len(copies) - 1)]
    stream = streams[0]
    torch.cuda.synchronize()
    if args.shapes:
        ctx.ft_set_shapes(*(int(v) for v in args.shapes.split(",")))
        shapes = ctx.ft_get_shapes()
    else:
        log("autotune")
        shapes = ctx.ft_autotune(jobs, stream=stream)
    torch.cuda.synchronize()

    pending = []
    n_streams = 1
    counter = [0]

    def submit_bounded():
        # keep at most max_inflight submissions outstanding (one ticket per
        # lane); consecutive submissions rotate over n_streams streams
        if len(pending) >= ctx.limits.max_inflight:
            ctx.ft_batch_wait(pending.pop(0))
        k = counter[0] % n_streams
        counter[0] += 1
        pending.append(ctx.ft_batch_submit(job_sets[k], streams[k]))

    def drain():
        while pending:
            ctx.ft_batch_wait(pending.pop(0))
        torch.cuda.synchronize()

    modes = {"graph": ft.FT_EXEC_GRAPH, "eager": ft.FT_EXEC_EAGER}
    trial = {}
    if args.exec == "auto" and not profiling:
        # submission streams: a short timed trial of each count
        for ns in range(1, max_streams + 1):
            ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
            n_streams = ns
            for _ in range(10):
                submit_bounded()
            drain()
            q0 = time.perf_counter()
            for _ in range(60):
                submit_bounded()
            drain()
            key = f"graph/s{ns}"
            trial[key] = round(n_frames * 60 / (time.perf_counter() - q0), 1)
            log("trial", key, trial[key])
        best = max(trial, key=trial.get)
        exec_mode, n_streams = "graph", int(best.split("/s")[1])
    elif profiling:
        exec_mode, n_streams = (args.exec if args.exec != "auto" else "graph"), 1
    else:
        exec_mode, n_streams = args.exec, args.streams
    ctx.ft_set_exec_mode(modes[exec_mode])

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        submit_bounded()
    drain()

    # ---- timed region: K back-to-back batch submissions, rotating over
    # n_streams streams (each with its own copy of the frames), so one batch's
    # latency-bound phases overlap the next one's search.
    log("timed", args.steps, exec_mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        submit_bounded()
    drain()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = n_frames * args.steps / dt
    if profiling:
        print(json.dumps({"workload": args.only, "value": round(value, 2), "ms_per_step": round(ms_per_step, 4),
                          "steps": args.steps, "exec": exec_mode}))
        return

    # ---- latency of one submission (submit -> completion seen by the host)
    lat = []
    for _ in range(max(50, args.steps // 4)):
        s0 = time.perf_counter()
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs, stream))
        lat.append((time.perf_counter() - s0) * 1e3)

    # ---- plain per-frame path on the same frames (single-frame calls)
    for d in dfs:
        d.run(ctx, stream)
    torch.cuda.synchronize()
    n_plain = max(5, args.steps // 10)
    p0 = time.perf_counter()
    for _ in range(n_plain):
        for d in dfs:
            d.run(ctx, stream)
    torch.cuda.synchronize()
    plain_fps = n_frames * n_plain / (time.perf_counter() - p0)

    # ---- per-kernel timing with HIP events on the launch stream, warm and
    # with the last-level cache flushed before every submission
    roofline, phases, phases_cold = None, None, None
    flush_buf = torch.empty(FLUSH_BYTES, dtype=torch.uint8, device="cuda")

    def flush():
        flush_buf.fill_(counter[0] & 0xFF)

    def one_submit():
        ctx.ft_batch_wait(ctx.ft_batch_submit(jobs, stream))

    if not args.no_timing:
        n_t = max(20, args.steps)
        phases = phase_times(ctx, ft, one_submit, n_t)
        phases_cold = phase_times(ctx, ft, one_submit, max(10, n_t // 2), flush=flush)
        ctx.ft_set_exec_mode(modes[exec_mode])
        dom = max(phases, key=lambda k: phases[k]["avg_us"] or 0)
        sbytes = algorithmic_search_bytes(frames)
        search_roof = search_roofline(sbytes, phases["search"]["avg_us"],
                                      measured_traffic("k_search_deal<JobTable>", "mixed_batch64"),
                                      "HIP events around each phase kernel, eager per-phase pass, warm caches")
        search_roof["dominant_phase"] = dom
        cold = search_roofline(sbytes, phases_cold["search"]["avg_us"], None,
                               "as warm, with a 512 MB write before every submission")
        search_roof["cold"] = {k: cold[k] for k in ("achieved", "frac", "avg_launch_us", "timed")}
        roofline = search_roof

    # ---- the three single-frame workloads: per-frame latency through the
    # single-frame calls (host wall time from the call to the stream's end)
    configs = None
    clustered = None
    if not args.no_extra:
        configs = {}
        reps = max(100, args.steps * 5)
        for name, f in single.items():
            d = ft.DeviceFrame(f, "cuda")
            for _ in range(10):
                d.run(ctx, stream)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                s0 = time.perf_counter()
                d.run(ctx, stream)
                stream.synchronize()
                ts.append((time.perf_counter() - s0) * 1e3)
            configs[name] = {**percentiles(ts), "frame_pairs_per_s": round(1e3 / float(np.mean(ts)), 1),
                             "reps": reps}
            log("single frame", name, configs[name])

        # ---- the clustered scene over 64 seeds in one submission
        log("clustered scene over 64 seeds")
        cframes = synth.clustered_batch()
        cdfs = [ft.DeviceFrame(f, "cuda") for f in cframes]
        cjobs = [d.job() for d in cdfs]
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
        for _ in range(5):
            ctx.ft_batch_wait(ctx.ft_batch_submit(cjobs, stream))
        torch.cuda.synchronize()
        csteps = max(20, args.steps)
        c0 = time.perf_counter()
        tickets = []
        for _ in range(csteps):
            if len(tickets) >= ctx.limits.max_inflight:
                ctx.ft_batch_wait(tickets.pop(0))
            tickets.append(ctx.ft_batch_submit(cjobs, stream))
        for t in tickets:
            ctx.ft_batch_wait(t)
        torch.cuda.synchronize()
        cdt = time.perf_counter() - c0
        clustered = {"workload": "clustered local map, 20000 map points in 40 blobs + 3000 keypoints, "
                                 "752x480 pinhole, 96x64 grid, 64 seeds, one submission per step",
                     "frame_pairs_per_s": round(len(cframes) * csteps / cdt, 1),
                     "ms_per_step": round(cdt * 1e3 / csteps, 4), "steps": csteps}
        if not args.no_timing:
            def csub():
                ctx.ft_batch_wait(ctx.ft_batch_submit(cjobs, stream))
            cph = phase_times(ctx, ft, csub, csteps)
            cph_cold = phase_times(ctx, ft, csub, max(10, csteps // 2), flush=flush)
            cb = algorithmic_search_bytes(cframes)
            croof = search_roofline(cb, cph["search"]["avg_us"],
                                    measured_traffic("k_search_deal<JobTable>", "clustered64"),
                                    "HIP events around each phase kernel, eager per-phase pass, warm caches")
            cold = search_roofline(cb, cph_cold["search"]["avg_us"], None,
                                   "as warm, with a 512 MB write before every submission")
            croof["cold"] = {k: cold[k] for k in ("achieved", "frac", "avg_launch_us", "timed")}
            clustered["phases"] = cph
            clustered["roofline"] = croof
        log("clustered", clustered["frame_pairs_per_s"], clustered.get("roofline", {}).get("frac"))
        ctx.ft_set_exec_mode(modes[exec_mode])
        del cdfs

    # ---- image pyramids built on the device: the same 64 frames with every
    # pinhole job building both of its pyramids before stereo (Section IV-B)
    pyramids = None
    last_frame = None
    if not args.no_extra:
        log("device pyramids")
        pdfs = [ft.DeviceFrame(f, "cuda", build_pyramids=True) for f in frames]
        pjobs = [d.job() for d in pdfs]
        ctx.ft_set_exec_mode(ft.FT_EXEC_GRAPH)
        for _ in range(5):
            ctx.ft_batch_wait(ctx.ft_batch_submit(pjobs, stream))
        torch.cuda.synchronize()
        psteps = max(20, args.steps)
        pt0 = time.perf_counter()
        tickets = []
        for _ in range(psteps):
            if len(tickets) >= ctx.limits.max_inflight:
                ctx.ft_batch_wait(tickets.pop(0))
            tickets.append(ctx.ft_batch_submit(pjobs, stream))
        for t in tickets:
            ctx.ft_batch_wait(t)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - pt0
        n_img = 2 * sum(d.build_pyramids for d in pdfs)
        pyramids = {"workload": "the benchmark's 64 frames, every pinhole job building both 8-level pyramids "
                                "(752x480 level 0) on the device before stereo",
                    "images_per_step": n_img,
                    "frame_pairs_per_s": round(len(frames) * psteps / pdt, 1), "steps": psteps}
        if not args.no_timing:
            def psub():
                ctx.ft_batch_wait(ctx.ft_batch_submit(pjobs, stream))
            pph = phase_times(ctx, ft, psub, psteps)
            pph_cold = phase_times(ctx, ft, psub, max(10, psteps // 2), flush=flush)
            # per image: level 0 read once, every level (level 0 included) written once
            pbytes = sum(int(d.pyr_left_t.numel()) + int(d.pyr_right_t.numel()) +
                         2 * int(d.pyr_left.width[0]) * int(d.pyr_left.height[0]) for d in pdfs if d.build_pyramids)
            proof = search_roofline(pbytes, pph["pyramid"]["avg_us"],
                                    measured_traffic("k_pyramid<JobTable>", "pyramids_batch64"),
                                    "HIP events around each phase kernel, eager per-phase pass, warm caches")
            proof["kernel"] = "k_pyramid (image pyramids)"
            cold = search_roofline(pbytes, pph_cold["pyramid"]["avg_us"], None,
                                   "as warm, with a 512 MB write before every submission")
            proof["cold"] = {k: cold[k] for k in ("achieved", "frac", "avg_launch_us", "timed")}
            pyramids["phases"] = pph
            pyramids["roofline"] = proof
        log("pyramids", pyramids["frame_pairs_per_s"], pyramids.get("roofline", {}).get("frac"))
        ctx.ft_set_exec_mode(modes[exec_mode])
        del pdfs, pjobs

        # ---- last-frame search by projection (Initial Pose Estimation):
        # single-frame calls on the pinhole and fisheye frames
        last_frame = {}
        for name in ("pinhole_frame_1200", "fisheye_frame_1500"):
            f = single[name]
            for view in range(len(f["search"])):
                case = synth.last_frame_case(f, 990 + view, view=view)
                dl = ft.DeviceLastFrame(case, "cuda")
                for _ in range(10):
                    dl.run(ctx, stream)
                torch.cuda.synchronize()
                reps = max(100, args.steps * 5)
                ts = []
                for _ in range(reps):
                    s0 = time.perf_counter()
                    dl.run(ctx, stream)
                    stream.synchronize()
                    ts.append((time.perf_counter() - s0) * 1e3)
                key = f"{name}/view{view}"
                last_frame[key] = {**percentiles(ts), "points": len(case["last"]["octave"]),
                                   "keypoints": len(case["kps"]["x"]),
                                   "calls_per_s": round(1e3 / float(np.mean(ts)), 1),
                                   "matches": dl.results()["n_matches"], "reps": reps}
                log("last frame", key, last_frame[key])

    # ---- ORB extraction on the device (Section II-A, IV-B)
    orb = None
    if not args.no_extra:
        log("orb extraction")
        orb = orb_leg(ctx, ft, frames, streams, args.steps, timing=not args.no_timing, flush=flush)
        log("orb", {k: v for k, v in orb.items() if k != "workload"})

    # ---- local-map maintenance on the device: a 20000-point map edited per
    # frame (5% of its points replaced; the kernels read the removal pairs and
    # the inserted points from pinned host memory) against uploading the whole
    # map again (one gather copy of its five arrays from pinned memory)
    map_maint = None
    if not args.no_extra:
        import ctypes as ct
        mf = synth.clustered_search_20000()[0]["map"]
        n_map, n_edit, cap = len(mf["dmin"]), 1000, 24000
        dmap = ft.DeviceMap(mf, cap)
        rng = np.random.default_rng(5)
        newp = synth.clustered_search_20000(seed=synth.seed_of(77))[0]["map"]
        keys = ("pos", "normal", "dmin", "dmax", "desc")

        def pinned_block(arrays):
            sizes = [-(-a.nbytes // 256) * 256 for a in arrays]
            base = ctx.ft_host_alloc(sum(sizes))
            view = np.ctypeslib.as_array((ct.c_uint8 * sum(sizes)).from_address(base))
            addrs, at = [], 0
            for a, sz in zip(arrays, sizes):
                view[at:at + a.nbytes] = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
                addrs.append(base + at)
                at += sz
            return base, addrs
        ins_base, ins_addr = pinned_block([newp[k][:n_edit] for k in keys])
        ins = ft.ft_map_points(n_edit, *ins_addr)
        whole_base, whole_addr = pinned_block([mf[k] for k in keys])
        whole_dev = {k: torch.empty(v.shape, dtype=torch.from_numpy(v[:1]).dtype, device="cuda") for k, v in mf.items()}
        segs = np.array([(whole_addr[i], whole_dev[k].data_ptr(), mf[k].nbytes) for i, k in enumerate(keys)],
                        dtype=np.int64)
        reps = max(200, args.steps)
        # removal lists drawn beforehand (the map size stays n_map)
        removals = [np.ascontiguousarray(rng.choice(n_map, n_edit, replace=False), dtype=np.int32)
                    for _ in range(reps + 10)]

        for k in range(10):
            ctx.ft_map_update(dmap.struct, cap, removals[reps + k], ins, stream=stream)
            ctx.ft_upload(segs, stream)
        torch.cuda.synchronize()
        te, tw = [], []
        for k in range(reps):
            s0 = time.perf_counter()
            ctx.ft_map_update(dmap.struct, cap, removals[k], ins, stream=stream)
            stream.synchronize()
            te.append((time.perf_counter() - s0) * 1e3)
        for _ in range(reps):
            s0 = time.perf_counter()
            ctx.ft_upload(segs, stream)
            stream.synchronize()
            tw.append((time.perf_counter() - s0) * 1e3)
        map_maint = {"workload": f"{n_map}-point local map, {n_edit} points removed and {n_edit} inserted per edit",
                     "edit_ms": percentiles(te), "whole_map_upload_ms": percentiles(tw),
                     "bytes_per_point": 64, "reps": reps,
                     "timed": "host clock around each edit (removal list, both kernels, inserted points read "
                              "from pinned memory) and each whole-map upload (one gather copy), synchronized"}
        log("map maintenance", map_maint)
        del dmap, whole_dev
        ctx.ft_host_free(ins_base)
        ctx.ft_host_free(whole_base)

    serving = None
    if args.serving > 0:
        del copies, dfs
        torch.cuda.empty_cache()
        serving = serving_sweep(args.serving, [2, 4, 8, 12, 16], [16, 64, 128, 192, 256, 384])

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "frame-pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "frames_per_step": n_frames,
                   "shapes": dict(zip(("best_lanes", "search_lanes", "aux_block"), shapes)),
                   "exec": exec_mode,
                   "submit_streams": n_streams, "exec_trial_fps": trial or None,
                   "pinhole_frames": sum(f["kind"] == "pinhole" for f in frames),
                   "fisheye_frames": sum(f["kind"] == "fisheye" for f in frames)},
        "latency_ms": {**percentiles(lat), "per": "64-frame submission"},
        "per_frame_path_fps": round(plain_fps, 2),
        "phases": phases,
        "phases_cold": phases_cold,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "single_frame_workloads": configs,
        "clustered_batch64": clustered,
        "device_pyramids": pyramids,
        "map_maintenance": map_maint,
        "orb_extraction": orb,
        "last_frame_search": last_frame,
        "serving": serving,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
