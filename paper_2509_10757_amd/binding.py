"""Python binding of libfasttrack (include/ft.h): argument marshalling only.

ctypes mirrors of the C structs, a `Context` whose methods carry the C entry
point names, and `DeviceFrame`, which places one synthetic frame's arrays in
device memory (torch tensors) and hands out the structs that point at them.
Every step of the hot path runs in the HIP library; if the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

from . import build as _build

LEVELS = 8
FT_OK, FT_ERR_INVALID_ARGUMENT, FT_ERR_CAPACITY, FT_ERR_DEVICE, FT_ERR_UNSUPPORTED = 0, 1, 2, 3, 4
FT_PHASES = 8
FT_CAMERA_PINHOLE, FT_CAMERA_KB = 0, 1
FT_JOB_PINHOLE, FT_JOB_FISHEYE, FT_JOB_SEARCH = 1, 2, 3
FT_EXEC_EAGER, FT_EXEC_GRAPH = 0, 1
FT_ORB_TESTS = 256
FT_PYRAMID_MAX_WIDTH = 1536

P = ct.c_void_p
F8 = ct.c_float * LEVELS


class ft_limits(ct.Structure):
    _fields_ = [("max_kp_per_image", ct.c_int32), ("max_map_points", ct.c_int32),
                ("max_rows", ct.c_int32), ("max_grid_cells", ct.c_int32),
                ("max_batch_frames", ct.c_int32), ("max_inflight", ct.c_int32),
                ("max_levels", ct.c_int32), ("max_batch_kp_total", ct.c_int32),
                ("max_batch_map_total", ct.c_int32)]


class ft_keypoints(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("x", P), ("y", P), ("octave", P), ("desc", P)]


class ft_pyramid(ct.Structure):
    _fields_ = [("data", P), ("offset", ct.c_int64 * LEVELS), ("width", ct.c_int32 * LEVELS),
                ("height", ct.c_int32 * LEVELS)]


class ft_scales(ct.Structure):
    _fields_ = [("n_levels", ct.c_int32), ("sf", F8), ("inv_sf", F8), ("sigma2", F8)]


class ft_pinhole_stereo(ct.Structure):
    _fields_ = [("fx", ct.c_float), ("bf", ct.c_float), ("b", ct.c_float), ("rows", ct.c_int32)]


class ft_pinhole_params(ct.Structure):
    _fields_ = [("th_orb", ct.c_int32), ("half_win", ct.c_int32), ("half_range", ct.c_int32),
                ("level_window", ct.c_int32), ("median_num", ct.c_int32),
                ("median_den", ct.c_int32), ("band", ct.c_float)]


class ft_pinhole_out(ct.Structure):
    _fields_ = [("right_idx", P), ("dist", P), ("u_right", P), ("depth", P), ("sad", P),
                ("n_matches", P)]


class ft_kb_intrinsics(ct.Structure):
    _fields_ = [("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("k", ct.c_float * 4)]


class ft_fisheye_stereo(ct.Structure):
    _fields_ = [("left", ft_kb_intrinsics), ("right", ft_kb_intrinsics), ("R_lr", ct.c_float * 9),
                ("t_lr", ct.c_float * 3), ("overlap_left", ct.c_float * 2),
                ("overlap_right", ct.c_float * 2)]


class ft_fisheye_params(ct.Structure):
    _fields_ = [("ratio_num", ct.c_int32), ("ratio_den", ct.c_int32), ("newton_iters", ct.c_int32),
                ("pad_", ct.c_int32), ("cos_parallax_max", ct.c_double), ("chi2", ct.c_double),
                ("max_theta", ct.c_double), ("newton_tol", ct.c_double)]


class ft_fisheye_out(ct.Structure):
    _fields_ = [("right_idx", P), ("dist", P), ("depth", P), ("xyz", P), ("n_matches", P)]


class ft_map_points(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("pos", P), ("normal", P), ("dmin", P), ("dmax", P),
                ("desc", P)]


class ft_search_camera(ct.Structure):
    _fields_ = [("model", ct.c_int32), ("fx", ct.c_float), ("fy", ct.c_float), ("cx", ct.c_float),
                ("cy", ct.c_float), ("k", ct.c_float * 4), ("bf", ct.c_float),
                ("R", ct.c_float * 9), ("t", ct.c_float * 3), ("O", ct.c_float * 3),
                ("min_x", ct.c_float), ("max_x", ct.c_float), ("min_y", ct.c_float),
                ("max_y", ct.c_float)]


class ft_grid(ct.Structure):
    _fields_ = [("cols", ct.c_int32), ("rows", ct.c_int32)]


class ft_search_params(ct.Structure):
    _fields_ = [("th", ct.c_float), ("view_cos_limit", ct.c_float), ("view_cos_narrow", ct.c_float),
                ("r_narrow", ct.c_float), ("r_wide", ct.c_float), ("dist_lo", ct.c_float),
                ("dist_hi", ct.c_float), ("level_lo", ct.c_int32), ("level_hi", ct.c_int32),
                ("th_high", ct.c_int32), ("ratio_num", ct.c_int32), ("ratio_den", ct.c_int32),
                ("ratio_same_level_only", ct.c_int32)]


class ft_search_out(ct.Structure):
    _fields_ = [("mp_match", P), ("mp_dist", P), ("kp_match", P), ("n_matches", P)]


class ft_orb_params(ct.Structure):
    _fields_ = [("threshold", ct.c_int32), ("edge", ct.c_int32)]


class ft_orb_corners(ct.Structure):
    _fields_ = [("capacity", ct.c_int32), ("lx", P), ("ly", P), ("octave", P), ("score", P), ("x", P), ("y", P),
                ("count", P)]


class ft_map_ids(ct.Structure):
    _fields_ = [("slot_id", P), ("slot_of", P), ("id_count", ct.c_int32)]


class ft_map_edit(ct.Structure):
    _fields_ = [("n_remove", ct.c_int32), ("remove", P), ("insert", ft_map_points), ("insert_ids", P),
                ("ids", ct.POINTER(ft_map_ids))]


class ft_image(ct.Structure):
    _fields_ = [("data", P), ("width", ct.c_int32), ("height", ct.c_int32), ("pitch", ct.c_int32)]


class ft_last_points(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("pos", P), ("desc", P), ("octave", P), ("angle", P)]


class ft_last_params(ct.Structure):
    _fields_ = [("th", ct.c_float), ("th_high", ct.c_int32), ("direction", ct.c_int32),
                ("check_orientation", ct.c_int32), ("bins", ct.c_int32)]


class ft_frame_job(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("n_views", ct.c_int32),
                ("left", ft_keypoints), ("right", ft_keypoints), ("scales", ft_scales),
                ("pyr_left", ft_pyramid), ("pyr_right", ft_pyramid),
                ("pinhole", ft_pinhole_stereo), ("pinhole_params", ft_pinhole_params),
                ("pinhole_out", ft_pinhole_out), ("use_u_right", ct.c_int32),
                ("build_pyramids", ct.c_int32), ("image_left", ft_image), ("image_right", ft_image),
                ("fisheye", ft_fisheye_stereo), ("fisheye_params", ft_fisheye_params),
                ("fisheye_out", ft_fisheye_out), ("map", ft_map_points),
                ("cam", ft_search_camera * 2), ("grid", ft_grid * 2), ("preassigned", P * 2),
                ("search_params", ft_search_params), ("search_out", ft_search_out * 2)]


class ft_segment(ct.Structure):
    _fields_ = [("src", P), ("dst", P), ("bytes", ct.c_int64)]


class ft_shapes(ct.Structure):
    _fields_ = [("best_lanes", ct.c_int32), ("search_lanes", ct.c_int32), ("aux_block", ct.c_int32)]


EXPORTS = {
    "ft_context_create": [ct.POINTER(ft_limits), ct.c_int32, ct.POINTER(P)],
    "ft_context_destroy": [P],
    "ft_context_workspace_bytes": [P, ct.POINTER(ct.c_int64)],
    "ft_stereo_match_pinhole": [P, P, ct.POINTER(ft_keypoints), ct.POINTER(ft_keypoints),
                                ct.POINTER(ft_pyramid), ct.POINTER(ft_pyramid), ct.POINTER(ft_scales),
                                ct.POINTER(ft_pinhole_stereo), ct.POINTER(ft_pinhole_params),
                                ct.POINTER(ft_pinhole_out)],
    "ft_stereo_match_fisheye": [P, P, ct.POINTER(ft_keypoints), ct.POINTER(ft_keypoints),
                                ct.POINTER(ft_scales), ct.POINTER(ft_fisheye_stereo),
                                ct.POINTER(ft_fisheye_params), ct.POINTER(ft_fisheye_out)],
    "ft_search_local_points": [P, P, ct.POINTER(ft_map_points), ct.POINTER(ft_search_camera),
                               ct.POINTER(ft_keypoints), P, P, ct.POINTER(ft_grid),
                               ct.POINTER(ft_scales), ct.POINTER(ft_search_params),
                               ct.POINTER(ft_search_out)],
    "ft_search_local_points_noalloc": [P, ct.POINTER(ft_map_points), ct.POINTER(ft_search_camera),
                                       ct.POINTER(ft_keypoints), P, P, ct.POINTER(ft_grid),
                                       ct.POINTER(ft_scales), ct.POINTER(ft_search_params),
                                       ct.POINTER(ft_search_out)],
    "ft_pyramid_layout": [ct.c_int32, ct.c_int32, ct.POINTER(ft_scales), ct.POINTER(ft_pyramid),
                          ct.POINTER(ct.c_int64)],
    "ft_build_pyramid": [P, P, ct.POINTER(ft_image), ct.POINTER(ft_scales), ct.POINTER(ft_pyramid)],
    "ft_search_last_frame": [P, P, ct.POINTER(ft_last_points), ct.POINTER(ft_search_camera),
                             ct.POINTER(ft_keypoints), P, P, P, ct.POINTER(ft_grid), ct.POINTER(ft_scales),
                             ct.POINTER(ft_last_params), ct.POINTER(ft_search_out)],
    "ft_map_update": [P, P, ct.POINTER(ft_map_points), ct.c_int32, ct.POINTER(ft_map_edit)],
    "ft_map_update_many": [P, P, ct.c_int32, ct.POINTER(ct.POINTER(ft_map_points)), P, ct.POINTER(ft_map_edit)],
    "ft_orb_detect": [P, P, ct.POINTER(ft_pyramid), ct.POINTER(ft_scales), ct.POINTER(ft_orb_params), P,
                      ct.POINTER(ft_orb_corners)],
    "ft_orb_describe": [P, P, ct.POINTER(ft_pyramid), P, ct.c_int32, P, P, P, P, P, P, P],
    "ft_batch_submit": [P, P, ct.POINTER(ft_frame_job), ct.c_int32, ct.POINTER(ct.c_uint64)],
    "ft_batch_poll": [P, ct.c_uint64, ct.POINTER(ct.c_int32)],
    "ft_batch_wait": [P, ct.c_uint64],
    "ft_context_enable_timing": [P, ct.c_int32],
    "ft_context_read_timing": [P, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)],
    "ft_set_exec_mode": [P, ct.c_int32],
    "ft_get_exec_mode": [P, ct.POINTER(ct.c_int32)],
    "ft_set_shapes": [P, ct.POINTER(ft_shapes)],
    "ft_get_shapes": [P, ct.POINTER(ft_shapes)],
    "ft_autotune": [P, P, ct.POINTER(ft_frame_job), ct.c_int32, ct.c_char_p, ct.POINTER(ft_shapes)],
    "ft_host_alloc": [P, ct.c_int64, ct.POINTER(P)],
    "ft_host_free": [P, P],
    "ft_upload": [P, P, ct.POINTER(ft_segment), ct.c_int32],
    "ft_status_string": [ct.c_int32],
    "ft_last_error": [P],
    "ft_version": [],
}

_lib = None


def library_path() -> str:
    return _build.LIB


def load():
    """Load libfasttrack.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it first (python -m paper_2509_10757_amd.build)")
        lib = ct.CDLL(path)
        for name, argtypes in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = ct.c_int32
        lib.ft_status_string.restype = ct.c_char_p
        lib.ft_last_error.restype = ct.c_char_p
        _lib = lib
    return _lib


class FtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def default_limits(**kw) -> ft_limits:
    v = dict(max_kp_per_image=4096, max_map_points=65536, max_rows=1024, max_grid_cells=8192,
             max_batch_frames=64, max_inflight=2, max_levels=LEVELS, max_batch_kp_total=0,
             max_batch_map_total=0)
    v.update(kw)
    return ft_limits(**v)


FT_NOALLOC_MAX_KP, FT_NOALLOC_MAX_MAP, FT_NOALLOC_SCRATCH_BYTES = 8192, 65536, 1 << 20


def ft_search_local_points_noalloc(map_points, cam, kps, u_right, preassigned, grid, scales, params,
                                   out, stream=None, check=True):
    """The context-free, allocation-free search (same outputs as
    Context.ft_search_local_points) on the current device."""
    lib = load()
    st = lib.ft_search_local_points_noalloc(_stream(stream), ct.byref(map_points), ct.byref(cam),
                                            ct.byref(kps), P(u_right or None), P(preassigned or None),
                                            ct.byref(grid), ct.byref(scales), ct.byref(params),
                                            ct.byref(out))
    if check and st != FT_OK:
        raise FtError(st, f"ft_search_local_points_noalloc: {lib.ft_last_error(None).decode()}")
    return st


def pyramid_layout(width: int, height: int, scales) -> tuple:
    """(ft_pyramid with offsets and sizes, total bytes) of a width x height
    image's pyramid, from the library."""
    lib = load()
    pyr = ft_pyramid()
    nb = ct.c_int64()
    st = lib.ft_pyramid_layout(width, height, ct.byref(scales), ct.byref(pyr), ct.byref(nb))
    if st != FT_OK:
        raise FtError(st, f"ft_pyramid_layout({width}, {height})")
    return pyr, nb.value


def _stream(stream) -> P:
    if stream is None:
        stream = torch.cuda.current_stream()
    return P(stream.cuda_stream)


class Context:
    """Owns an ft_context; methods carry the C entry point names."""

    def __init__(self, limits: ft_limits | None = None, device: int = 0):
        self.lib = load()
        self.limits = limits or default_limits()
        h = P()
        st = self.lib.ft_context_create(ct.byref(self.limits), device, ct.byref(h))
        if st != FT_OK:
            raise FtError(st, f"ft_context_create failed: {self.lib.ft_status_string(st).decode()}")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.ft_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != FT_OK:
            raise FtError(st, f"{what}: {self.lib.ft_last_error(self.h).decode()}")

    def workspace_bytes(self) -> int:
        v = ct.c_int64()
        self._check(self.lib.ft_context_workspace_bytes(self.h, ct.byref(v)), "workspace_bytes")
        return v.value

    PHASES = ("pyramid", "setup", "stereo_best", "pinhole_refine", "fisheye_triangulate", "stereo_resolve",
              "search", "search_resolve")

    def ft_context_enable_timing(self, enable: bool = True):
        self._check(self.lib.ft_context_enable_timing(self.h, int(enable)), "enable_timing")

    def ft_context_read_timing(self) -> dict:
        ms = (ct.c_double * FT_PHASES)()
        n = (ct.c_int64 * FT_PHASES)()
        self._check(self.lib.ft_context_read_timing(self.h, ms, n), "read_timing")
        return {p: (ms[i], n[i]) for i, p in enumerate(self.PHASES)}

    def ft_stereo_match_pinhole(self, left, right, pyr_left, pyr_right, scales, cam, params, out,
                                stream=None, check=True):
        st = self.lib.ft_stereo_match_pinhole(self.h, _stream(stream), ct.byref(left), ct.byref(right),
                                              ct.byref(pyr_left), ct.byref(pyr_right), ct.byref(scales),
                                              ct.byref(cam), ct.byref(params), ct.byref(out))
        if check:
            self._check(st, "ft_stereo_match_pinhole")
        return st

    def ft_stereo_match_fisheye(self, left, right, scales, cam, params, out, stream=None, check=True):
        st = self.lib.ft_stereo_match_fisheye(self.h, _stream(stream), ct.byref(left), ct.byref(right),
                                              ct.byref(scales), ct.byref(cam), ct.byref(params),
                                              ct.byref(out))
        if check:
            self._check(st, "ft_stereo_match_fisheye")
        return st

    def ft_search_local_points(self, map_points, cam, kps, u_right, preassigned, grid, scales,
                               params, out, stream=None, check=True):
        st = self.lib.ft_search_local_points(self.h, _stream(stream), ct.byref(map_points),
                                             ct.byref(cam), ct.byref(kps), P(u_right or None),
                                             P(preassigned or None), ct.byref(grid), ct.byref(scales),
                                             ct.byref(params), ct.byref(out))
        if check:
            self._check(st, "ft_search_local_points")
        return st

    def ft_build_pyramid(self, image, scales, pyr, stream=None, check=True):
        st = self.lib.ft_build_pyramid(self.h, _stream(stream), ct.byref(image), ct.byref(scales), ct.byref(pyr))
        if check:
            self._check(st, "ft_build_pyramid")
        return st

    def ft_search_last_frame(self, last, cam, kps, kp_angle, u_right, preassigned, grid, scales, params, out,
                             stream=None, check=True):
        st = self.lib.ft_search_last_frame(self.h, _stream(stream), ct.byref(last), ct.byref(cam), ct.byref(kps),
                                           P(kp_angle or None), P(u_right or None), P(preassigned or None),
                                           ct.byref(grid), ct.byref(scales), ct.byref(params), ct.byref(out))
        if check:
            self._check(st, "ft_search_last_frame")
        return st

    def ft_map_update(self, map_points, capacity: int, remove, insert, stream=None, check=True, ids=None,
                      insert_ids=None):
        """Edit a device map in place; `map_points.n` is updated.  `remove`:
        host slot indices (a sequence), or point ids when `ids` (an
        ft_map_ids record, kept by the call) is given; `insert`: an
        ft_map_points of device or ft_host_alloc arrays (or None);
        `insert_ids`: the inserted points' ids (with `ids`)."""
        rem = np.ascontiguousarray(np.asarray(remove, dtype=np.int32).reshape(-1))
        iid = None if insert_ids is None else np.ascontiguousarray(np.asarray(insert_ids, dtype=np.int32))
        ed = ft_map_edit(len(rem), P(rem.ctypes.data if len(rem) else None),
                         insert if insert is not None else ft_map_points(),
                         P(iid.ctypes.data if iid is not None and len(iid) else None),
                         ct.pointer(ids) if ids is not None else None)
        st = self.lib.ft_map_update(self.h, _stream(stream), ct.byref(map_points), capacity, ct.byref(ed))
        if check:
            self._check(st, "ft_map_update")
        return st

    def ft_map_update_many(self, maps, capacities, edits, stream=None, check=True):
        """Edits of several distinct maps in one call: `maps` a sequence of
        ft_map_points (each one's n updated), `capacities` ints, `edits`
        ft_map_edit structs (arrays they point to kept alive by the caller)."""
        n = len(maps)
        mp = (ct.POINTER(ft_map_points) * max(n, 1))(*[ct.pointer(m) for m in maps])
        cap = np.ascontiguousarray(np.asarray(capacities, dtype=np.int32))
        ed = (ft_map_edit * max(n, 1))(*edits)
        st = self.lib.ft_map_update_many(self.h, _stream(stream), n, mp, P(cap.ctypes.data if n else None), ed)
        if check:
            self._check(st, "ft_map_update_many")
        return st

    def ft_map_update_raw(self, map_points, capacity: int, edit, stream):
        """ft_map_update with a prepared ft_map_edit (arrays kept alive by
        the caller): one call, no conversions."""
        return self._check(self.lib.ft_map_update(self.h, P(stream.cuda_stream), ct.byref(map_points), capacity,
                                                  ct.byref(edit)), "ft_map_update")

    def ft_orb_detect(self, pyr, scales, params, blurred, corners, stream=None, check=True):
        """`blurred`: device address or None; `corners`: ft_orb_corners."""
        st = self.lib.ft_orb_detect(self.h, _stream(stream), ct.byref(pyr), ct.byref(scales), ct.byref(params),
                                    P(blurred or None), ct.byref(corners))
        if check:
            self._check(st, "ft_orb_detect")
        return st

    def ft_orb_describe(self, pyr, blurred, n_max, count, lx, ly, octave, pattern, angle, desc, stream=None,
                        check=True):
        """Device addresses (count may be None); `pattern`: host int8 [256, 4]."""
        pat = np.ascontiguousarray(np.asarray(pattern, dtype=np.int8).reshape(-1))
        st = self.lib.ft_orb_describe(self.h, _stream(stream), ct.byref(pyr), P(blurred or None), int(n_max),
                                      P(count or None), P(lx or None), P(ly or None), P(octave or None),
                                      P(pat.ctypes.data), P(angle or None), P(desc or None))
        if check:
            self._check(st, "ft_orb_describe")
        return st

    def ft_batch_submit(self, jobs, stream=None) -> int:
        arr = (ft_frame_job * len(jobs))(*jobs)
        t = ct.c_uint64()
        self._check(self.lib.ft_batch_submit(self.h, _stream(stream), arr, len(jobs), ct.byref(t)),
                    "ft_batch_submit")
        return t.value

    def ft_batch_submit_raw(self, addr: int, n: int, stream=None) -> int:
        """Submit `n` jobs already laid out as ft_frame_job structs at host
        address `addr` (e.g. a NumPy buffer)."""
        t = ct.c_uint64()
        arr = ct.cast(P(addr), ct.POINTER(ft_frame_job))
        self._check(self.lib.ft_batch_submit(self.h, _stream(stream), arr, n, ct.byref(t)), "ft_batch_submit")
        return t.value

    def ft_host_alloc(self, nbytes: int) -> int:
        p = P()
        self._check(self.lib.ft_host_alloc(self.h, nbytes, ct.byref(p)), "ft_host_alloc")
        return p.value

    def ft_host_free(self, addr: int):
        self._check(self.lib.ft_host_free(self.h, P(addr)), "ft_host_free")

    def ft_upload(self, segs, stream=None, check=True):
        """`segs`: a C-contiguous int64 array of shape (n, 3) holding (src,
        dst, bytes) rows, or a sequence of such triples."""
        a = np.ascontiguousarray(np.asarray(segs, dtype=np.int64).reshape(-1, 3))
        st = self.lib.ft_upload(self.h, _stream(stream), ct.cast(P(a.ctypes.data), ct.POINTER(ft_segment)),
                                len(a))
        if check:
            self._check(st, "ft_upload")
        return st

    def ft_set_exec_mode(self, mode: int):
        self._check(self.lib.ft_set_exec_mode(self.h, mode), "ft_set_exec_mode")

    def ft_get_exec_mode(self) -> int:
        m = ct.c_int32()
        self._check(self.lib.ft_get_exec_mode(self.h, ct.byref(m)), "ft_get_exec_mode")
        return m.value

    def ft_set_shapes(self, best_lanes: int, search_lanes: int, aux_block: int = 1024):
        sh = ft_shapes(best_lanes, search_lanes, aux_block)
        self._check(self.lib.ft_set_shapes(self.h, ct.byref(sh)), "ft_set_shapes")

    def ft_get_shapes(self) -> tuple:
        s = ft_shapes()
        self._check(self.lib.ft_get_shapes(self.h, ct.byref(s)), "ft_get_shapes")
        return s.best_lanes, s.search_lanes, s.aux_block

    def ft_autotune(self, jobs, cache_path=None, stream=None) -> tuple:
        arr = (ft_frame_job * len(jobs))(*jobs)
        s = ft_shapes()
        cp = cache_path.encode() if cache_path else None
        self._check(self.lib.ft_autotune(self.h, _stream(stream), arr, len(jobs), cp, ct.byref(s)),
                    "ft_autotune")
        return s.best_lanes, s.search_lanes, s.aux_block

    def ft_batch_poll(self, ticket: int) -> bool:
        d = ct.c_int32()
        self._check(self.lib.ft_batch_poll(self.h, ct.c_uint64(ticket), ct.byref(d)), "ft_batch_poll")
        return bool(d.value)

    def ft_batch_wait(self, ticket: int):
        self._check(self.lib.ft_batch_wait(self.h, ct.c_uint64(ticket)), "ft_batch_wait")


# --------------------------------------------------------------------------
# Device placement of one synthetic frame
# --------------------------------------------------------------------------
def _dev(a, dtype=None, device="cuda"):
    t = torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype)))
    return t.to(device)


def _ptr(t):
    return t.data_ptr() if t is not None and t.numel() > 0 else None


def _scales(sc) -> ft_scales:
    s = ft_scales()
    s.n_levels = LEVELS
    s.sf[:] = [float(v) for v in sc["sf"]]
    s.inv_sf[:] = [float(v) for v in sc["inv_sf"]]
    s.sigma2[:] = [float(v) for v in sc["sigma2"]]
    return s


class DeviceKeypoints:
    def __init__(self, kp, device):
        self.n = len(kp["x"])
        self.x = _dev(kp["x"], np.float32, device)
        self.y = _dev(kp["y"], np.float32, device)
        self.octave = _dev(kp["octave"], np.uint8, device)
        self.desc = _dev(kp["desc"], np.uint8, device)

    def struct(self) -> ft_keypoints:
        return ft_keypoints(self.n, _ptr(self.x), _ptr(self.y), _ptr(self.octave), _ptr(self.desc))


def _pyramid(pyr, device):
    t = _dev(pyr["data"], np.uint8, device)
    s = ft_pyramid()
    s.data = _ptr(t)
    s.offset[:] = [int(v) for v in pyr["offset"]]
    s.width[:] = [int(v) for v in pyr["width"]]
    s.height[:] = [int(v) for v in pyr["height"]]
    return t, s


def _kb(c) -> ft_kb_intrinsics:
    k = ft_kb_intrinsics(float(c["fx"]), float(c["fy"]), float(c["cx"]), float(c["cy"]))
    k.k[:] = [float(v) for v in c["k"]]
    return k


def search_camera_struct(cam) -> ft_search_camera:
    s = ft_search_camera()
    s.model = int(cam["model"])
    s.fx, s.fy, s.cx, s.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    s.k[:] = [float(v) for v in cam["k"]]
    s.bf = float(cam["bf"])
    s.R[:] = [float(v) for v in np.asarray(cam["R"], np.float32).reshape(-1)]
    s.t[:] = [float(v) for v in cam["t"]]
    s.O[:] = [float(v) for v in cam["O"]]
    s.min_x, s.max_x, s.min_y, s.max_y = (float(v) for v in cam["bounds"])
    return s


def search_params_struct(sp) -> ft_search_params:
    return ft_search_params(sp["th"], sp["view_cos_limit"], sp["view_cos_narrow"], sp["r_narrow"],
                            sp["r_wide"], sp["dist_lo"], sp["dist_hi"], sp["level_lo"], sp["level_hi"],
                            sp["th_high"], sp["ratio_num"], sp["ratio_den"], sp["ratio_same_level_only"])


class DeviceFrame:
    """One synthetic frame resident in device memory, with output buffers."""

    def __init__(self, frame: dict, device="cuda", build_pyramids: bool = False):
        """build_pyramids (pinhole): upload only level 0 of each image and let
        the batch job build both pyramids on the device before stereo (the
        pyramid buffers start filled with 0xA5)."""
        self.frame = frame
        self.kind = frame["kind"]
        self.device = device
        self.left = DeviceKeypoints(frame["left"], device)
        self.right = DeviceKeypoints(frame["right"], device) if "right" in frame else None
        self.scales = _scales(frame["scales"])
        self.build_pyramids = bool(build_pyramids) and self.kind == "pinhole"
        nL = self.left.n
        i32 = dict(dtype=torch.int32, device=device)
        f32 = dict(dtype=torch.float32, device=device)
        if self.kind == "pinhole" and self.build_pyramids:
            self.images = {}
            for side in ("left", "right"):
                pyr = frame["pyr_" + side]
                w, h = int(pyr["width"][0]), int(pyr["height"][0])
                img_t = _dev(pyr["data"][:w * h], np.uint8, device)
                lay, nbytes = pyramid_layout(w, h, self.scales)
                out_t = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device=device)
                lay.data = _ptr(out_t)
                self.images[side] = (img_t, ft_image(_ptr(img_t), w, h, w))
                setattr(self, "pyr_%s_t" % side, out_t)
                setattr(self, "pyr_" + side, lay)
        if self.kind == "pinhole":
            if not self.build_pyramids:
                self.pyr_left_t, self.pyr_left = _pyramid(frame["pyr_left"], device)
                self.pyr_right_t, self.pyr_right = _pyramid(frame["pyr_right"], device)
            c, sp = frame["stereo_cam"], frame["stereo_params"]
            self.stereo_cam = ft_pinhole_stereo(float(c["fx"]), float(c["bf"]), float(c["b"]), int(c["rows"]))
            self.stereo_params = ft_pinhole_params(sp["th_orb"], sp["half_win"], sp["half_range"],
                                                   sp["level_window"], sp["median_num"],
                                                   sp["median_den"], sp["band"])
            self.o = {"right_idx": torch.empty(nL, **i32), "dist": torch.empty(nL, **i32),
                      "u_right": torch.empty(nL, **f32), "depth": torch.empty(nL, **f32),
                      "sad": torch.empty(nL, **i32), "n_matches": torch.empty(1, **i32)}
            o = self.o
            self.stereo_out = ft_pinhole_out(_ptr(o["right_idx"]), _ptr(o["dist"]), _ptr(o["u_right"]),
                                             _ptr(o["depth"]), _ptr(o["sad"]), _ptr(o["n_matches"]))
        elif self.kind == "fisheye":
            c, sp = frame["stereo_cam"], frame["stereo_params"]
            fs = ft_fisheye_stereo()
            fs.left, fs.right = _kb(c["left"]), _kb(c["right"])
            fs.R_lr[:] = [float(v) for v in np.asarray(c["R_lr"], np.float32).reshape(-1)]
            fs.t_lr[:] = [float(v) for v in c["t_lr"]]
            fs.overlap_left[:] = [float(v) for v in c["overlap_left"]]
            fs.overlap_right[:] = [float(v) for v in c["overlap_right"]]
            self.stereo_cam = fs
            self.stereo_params = ft_fisheye_params(sp["ratio_num"], sp["ratio_den"], sp["newton_iters"], 0,
                                                   sp["cos_parallax_max"], sp["chi2"],
                                                   float(np.deg2rad(sp["max_theta_deg"])), sp["newton_tol"])
            self.o = {"right_idx": torch.empty(nL, **i32), "dist": torch.empty(nL, **i32),
                      "depth": torch.empty(nL, **f32), "xyz": torch.empty((nL, 3), **f32),
                      "n_matches": torch.empty(1, **i32)}
            o = self.o
            self.stereo_out = ft_fisheye_out(_ptr(o["right_idx"]), _ptr(o["dist"]), _ptr(o["depth"]),
                                             _ptr(o["xyz"]), _ptr(o["n_matches"]))
        mp = frame["map"]
        self.nM = len(mp["dmin"])
        self.map_t = {"pos": _dev(mp["pos"], np.float32, device), "normal": _dev(mp["normal"], np.float32, device),
                      "dmin": _dev(mp["dmin"], np.float32, device), "dmax": _dev(mp["dmax"], np.float32, device),
                      "desc": _dev(mp["desc"], np.uint8, device)}
        m = self.map_t
        self.map = ft_map_points(self.nM, _ptr(m["pos"]), _ptr(m["normal"]), _ptr(m["dmin"]),
                                 _ptr(m["dmax"]), _ptr(m["desc"]))
        self.search_params = search_params_struct(frame["search_params"])
        self.views = []
        for spec in frame["search"]:
            kps = self.left if spec["image"] == "left" else self.right
            pre = spec.get("preassigned")
            pre_t = _dev(pre, np.uint8, device) if pre is not None else None
            out = {"mp_match": torch.empty(self.nM, **i32), "mp_dist": torch.empty(self.nM, **i32),
                   "kp_match": torch.empty(kps.n, **i32), "n_matches": torch.empty(1, **i32)}
            self.views.append({
                "kps": kps, "cam": search_camera_struct(spec["cam"]),
                "grid": ft_grid(*spec["grid"]), "pre_t": pre_t, "out_t": out,
                "out": ft_search_out(_ptr(out["mp_match"]), _ptr(out["mp_dist"]), _ptr(out["kp_match"]),
                                     _ptr(out["n_matches"])),
                "use_u_right": bool(spec.get("use_u_right")) and self.kind == "pinhole",
            })

    # -- the per-frame path: one C call per step, in order on one stream
    def run(self, ctx: Context, stream=None, u_right=None):
        if self.kind == "pinhole":
            ctx.ft_stereo_match_pinhole(self.left.struct(), self.right.struct(), self.pyr_left,
                                        self.pyr_right, self.scales, self.stereo_cam, self.stereo_params,
                                        self.stereo_out, stream=stream)
        elif self.kind == "fisheye":
            ctx.ft_stereo_match_fisheye(self.left.struct(), self.right.struct(), self.scales,
                                        self.stereo_cam, self.stereo_params, self.stereo_out, stream=stream)
        for v in self.views:
            ur = None
            if v["use_u_right"]:
                ur = _ptr(self.o["u_right"])
            elif u_right is not None:
                ur = _ptr(u_right)
            ctx.ft_search_local_points(self.map, v["cam"], v["kps"].struct(), ur, _ptr(v["pre_t"]),
                                       v["grid"], self.scales, self.search_params, v["out"], stream=stream)

    def job(self, stereo: bool = True) -> ft_frame_job:
        """The frame as a batch job; stereo=False submits its search views only
        (a search job, for frames whose views need no stereo output)."""
        j = ft_frame_job()
        kind = self.kind if stereo else "search"
        j.kind = {"pinhole": FT_JOB_PINHOLE, "fisheye": FT_JOB_FISHEYE}.get(kind, FT_JOB_SEARCH)
        j.n_views = len(self.views)
        j.left = self.left.struct()
        if self.right is not None:
            j.right = self.right.struct()
        j.scales = self.scales
        if kind == "pinhole":
            j.pyr_left, j.pyr_right = self.pyr_left, self.pyr_right
            if self.build_pyramids:
                j.build_pyramids = 1
                j.image_left, j.image_right = self.images["left"][1], self.images["right"][1]
            j.pinhole, j.pinhole_params, j.pinhole_out = self.stereo_cam, self.stereo_params, self.stereo_out
            j.use_u_right = int(self.views[0]["use_u_right"]) if self.views else 0
        elif kind == "fisheye":
            j.fisheye, j.fisheye_params, j.fisheye_out = self.stereo_cam, self.stereo_params, self.stereo_out
        j.map = self.map
        for i, v in enumerate(self.views):
            j.cam[i] = v["cam"]
            j.grid[i] = v["grid"]
            j.preassigned[i] = _ptr(v["pre_t"])
            j.search_out[i] = v["out"]
        j.search_params = self.search_params
        return j

    def pyramids(self) -> dict:
        """The pinhole pyramid buffers as host arrays (synchronises)."""
        return {side: getattr(self, "pyr_%s_t" % side).cpu().numpy() for side in ("left", "right")}

    def results(self) -> dict:
        """Copy every output to host numpy arrays (synchronises)."""
        res = {"kind": self.kind}
        if self.kind in ("pinhole", "fisheye"):
            st = {k: v.cpu().numpy() for k, v in self.o.items()}
            st["n_matches"] = int(st["n_matches"][0])
            res["stereo"] = st
        res["search"] = []
        for v in self.views:
            s = {k: t.cpu().numpy() for k, t in v["out_t"].items()}
            s["n_matches"] = int(s["n_matches"][0])
            res["search"].append(s)
        return res


class DeviceLastFrame:
    """A last-frame search case (synth.last_frame_case) resident in device
    memory, with output buffers."""

    def __init__(self, case: dict, device="cuda"):
        last, kps, prm = case["last"], case["kps"], case["params"]
        self.n = len(last["octave"])
        self.t = {"pos": _dev(last["pos"], np.float32, device), "desc": _dev(last["desc"], np.uint8, device),
                  "octave": _dev(last["octave"], np.uint8, device), "angle": _dev(last["angle"], np.float32, device),
                  "kp_angle": _dev(kps["angle"], np.float32, device)}
        self.kps = DeviceKeypoints(kps, device)
        self.u_right = None if case.get("u_right") is None else _dev(case["u_right"], np.float32, device)
        self.pre = None if case.get("preassigned") is None else _dev(case["preassigned"], np.uint8, device)
        t = self.t
        self.last = ft_last_points(self.n, _ptr(t["pos"]), _ptr(t["desc"]), _ptr(t["octave"]), _ptr(t["angle"]))
        self.cam = search_camera_struct(case["cam"])
        self.grid = ft_grid(*case["grid"])
        self.scales = _scales(case["scales"])
        self.params = ft_last_params(float(prm["th"]), int(prm["th_high"]), int(prm["direction"]),
                                     int(prm["check_orientation"]), int(prm["bins"]))
        i32 = dict(dtype=torch.int32, device=device)
        self.o = {"mp_match": torch.full((self.n,), -7, **i32), "mp_dist": torch.full((self.n,), -7, **i32),
                  "kp_match": torch.full((self.kps.n,), -7, **i32), "n_matches": torch.full((1,), -7, **i32)}
        o = self.o
        self.out = ft_search_out(_ptr(o["mp_match"]), _ptr(o["mp_dist"]), _ptr(o["kp_match"]), _ptr(o["n_matches"]))

    def run(self, ctx: Context, stream=None, check=True):
        return ctx.ft_search_last_frame(self.last, self.cam, self.kps.struct(), _ptr(self.t["kp_angle"]),
                                        _ptr(self.u_right), _ptr(self.pre), self.grid, self.scales, self.params,
                                        self.out, stream=stream, check=check)

    def results(self) -> dict:
        r = {k: v.cpu().numpy() for k, v in self.o.items()}
        return {"last_match": r["mp_match"], "last_dist": r["mp_dist"], "kp_match": r["kp_match"],
                "n_matches": int(r["n_matches"][0])}


class DeviceOrb:
    """ORB extraction of one device pyramid: the smoothed pyramid and corner
    outputs (capacity corners) allocated once; detect() then describe() run
    on the device with no host round trip (describe reads the device count)."""

    def __init__(self, pyr: dict, capacity: int = 65536, device="cuda"):
        n = int(pyr["data"].size) if isinstance(pyr["data"], np.ndarray) else int(pyr["data"].numel())
        self.pyr_t = pyr["data"] if isinstance(pyr["data"], torch.Tensor) else \
            torch.from_numpy(np.ascontiguousarray(pyr["data"])).to(device)
        self.pyr = ft_pyramid()
        self.pyr.data = self.pyr_t.data_ptr()
        self.pyr.offset[:] = [int(v) for v in pyr["offset"]]
        self.pyr.width[:] = [int(v) for v in pyr["width"]]
        self.pyr.height[:] = [int(v) for v in pyr["height"]]
        self.blurred = torch.empty(n, dtype=torch.uint8, device=device)
        self.capacity = capacity
        c = capacity
        self.t = {"lx": torch.empty(c, dtype=torch.int16, device=device),
                  "ly": torch.empty(c, dtype=torch.int16, device=device),
                  "octave": torch.empty(c, dtype=torch.uint8, device=device),
                  "score": torch.empty(c, dtype=torch.uint8, device=device),
                  "x": torch.empty(c, dtype=torch.float32, device=device),
                  "y": torch.empty(c, dtype=torch.float32, device=device),
                  "count": torch.zeros(1, dtype=torch.int32, device=device),
                  "angle": torch.empty(c, dtype=torch.float32, device=device),
                  "desc": torch.empty((c, 32), dtype=torch.uint8, device=device)}
        t = self.t
        self.corners = ft_orb_corners(c, _ptr(t["lx"]), _ptr(t["ly"]), _ptr(t["octave"]), _ptr(t["score"]),
                                      _ptr(t["x"]), _ptr(t["y"]), _ptr(t["count"]))

    def detect(self, ctx: Context, scales, threshold=20, edge=19, stream=None, check=True):
        return ctx.ft_orb_detect(self.pyr, scales, ft_orb_params(threshold, edge), self.blurred.data_ptr(),
                                 self.corners, stream=stream, check=check)

    def describe(self, ctx: Context, pattern, stream=None, check=True):
        t = self.t
        return ctx.ft_orb_describe(self.pyr, self.blurred.data_ptr(), self.capacity, _ptr(t["count"]),
                                   _ptr(t["lx"]), _ptr(t["ly"]), _ptr(t["octave"]), pattern, _ptr(t["angle"]),
                                   _ptr(t["desc"]), stream=stream, check=check)

    def results(self) -> dict:
        n = int(self.t["count"][0])
        k = min(n, self.capacity)
        out = {key: self.t[key][:k].cpu().numpy() for key in ("lx", "ly", "octave", "score", "x", "y", "angle",
                                                                "desc")}
        out["count"] = n
        return out


class DeviceMap:
    """A local map in device memory with room for `capacity` points, edited in
    place with ft_map_update."""

    def __init__(self, mp: dict, capacity: int, device="cuda"):
        n = len(mp["dmin"])
        self.capacity = capacity
        self.t = {"pos": torch.zeros((capacity, 3), dtype=torch.float32, device=device),
                  "normal": torch.zeros((capacity, 3), dtype=torch.float32, device=device),
                  "dmin": torch.zeros(capacity, dtype=torch.float32, device=device),
                  "dmax": torch.zeros(capacity, dtype=torch.float32, device=device),
                  "desc": torch.zeros((capacity, 32), dtype=torch.uint8, device=device)}
        for k, v in self.t.items():
            if n:
                v[:n] = _dev(mp[k], v.cpu().numpy().dtype, device)
        t = self.t
        self.struct = ft_map_points(n, _ptr(t["pos"]), _ptr(t["normal"]), _ptr(t["dmin"]), _ptr(t["dmax"]),
                                    _ptr(t["desc"]))

    @property
    def n(self) -> int:
        return self.struct.n

    def edit(self, ctx: Context, remove, insert: dict | None, stream=None, check=True):
        """Remove host indices `remove` and append the points of host dict
        `insert` (uploaded first)."""
        ins = None
        self._ins = None
        if insert is not None and len(insert["dmin"]):
            self._ins = {k: _dev(np.ascontiguousarray(v), None, self.t[k].device) for k, v in insert.items()}
            i = self._ins
            ins = ft_map_points(len(insert["dmin"]), _ptr(i["pos"]), _ptr(i["normal"]), _ptr(i["dmin"]),
                                _ptr(i["dmax"]), _ptr(i["desc"]))
        return ctx.ft_map_update(self.struct, self.capacity, remove, ins, stream=stream, check=check)

    def host(self) -> dict:
        n = self.n
        return {k: v[:n].cpu().numpy() for k, v in self.t.items()}
