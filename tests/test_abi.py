"""The C ABI library loads and exports every entry point that include/ft.h
declares, and the binding's ctypes structs have the C compiler's layout.
No compute call is made (no GPU needed)."""
import ctypes as ct
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ft.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ft_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2509_10757_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return ct.CDLL(build.LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_2509_10757_amd import binding
    assert set(declared_functions()) == set(binding.EXPORTS)


def test_status_strings_without_device(lib):
    lib.ft_status_string.restype = ct.c_char_p
    assert lib.ft_status_string(0) == b"ok"
    assert lib.ft_status_string(2) == b"capacity exceeded"
    assert lib.ft_status_string(4) == b"unsupported"
    assert lib.ft_status_string(5) == b"unknown status"
    lib.ft_version.restype = ct.c_int32
    assert lib.ft_version() >= 100


STRUCTS = ["ft_limits", "ft_keypoints", "ft_pyramid", "ft_scales", "ft_pinhole_stereo",
           "ft_pinhole_params", "ft_pinhole_out", "ft_kb_intrinsics", "ft_fisheye_stereo",
           "ft_fisheye_params", "ft_fisheye_out", "ft_map_points", "ft_search_camera", "ft_grid",
           "ft_search_params", "ft_search_out", "ft_frame_job", "ft_shapes", "ft_image", "ft_last_points",
           "ft_last_params", "ft_map_edit", "ft_map_ids", "ft_orb_params", "ft_orb_corners"]


def test_ctypes_layout_matches_c_compiler(tmp_path):
    from paper_2509_10757_amd import binding
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ft.h"', 'int main(void){']
    for s in STRUCTS:
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for name, _ in getattr(binding, s)._fields_:
            lines.append(f'printf("{s}.{name} %zu\\n", offsetof({s}, {name}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in out:
        if not line:
            continue
        key, val = line.split()
        if "." in key:
            s, f = key.split(".")
            assert getattr(getattr(binding, s), f).offset == int(val), key
        else:
            assert ct.sizeof(getattr(binding, key)) == int(val), key


def test_binding_constants_match_header():
    """Every #define of the header that the binding mirrors has the same value
    (the timing arrays are sized by FT_PHASES, so a mismatch overruns them)."""
    from paper_2509_10757_amd import binding
    defs = dict(re.findall(r"#define\s+(FT_[A-Z_0-9]+)\s+(-?\d+)", open(HEADER).read()))
    mirrored = [k for k in defs if hasattr(binding, k)]
    assert {"FT_PHASES", "FT_EXEC_GRAPH", "FT_ERR_DEVICE"} <= set(mirrored)
    for k in mirrored:
        assert getattr(binding, k) == int(defs[k]), k
    assert len(binding.Context.PHASES) == int(defs["FT_PHASES"])
