"""Element-by-element comparison of device results with the CPU oracle.

Indices and Hamming distances must be bit-identical.  Sub-pixel right
coordinates must agree within 1e-5 px and depths within 1e-6 relative (the
float tolerance of the matching contract); fisheye points within 1e-6 of their
norm (float64 with libm vs the device math library, rounded to float32).
"""
import numpy as np

UR_TOL_PX = 1e-5
REL_TOL = 1e-6


def _eq(a, b, what):
    a = np.asarray(a); b = np.asarray(b)
    assert a.shape == b.shape, f"{what}: shape {a.shape} vs {b.shape}"
    bad = np.nonzero(a != b)[0]
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5].tolist()}: got {a[bad[:5]].tolist()} want {b[bad[:5]].tolist()}"


def compare_stereo(kind, got, want):
    _eq(got["right_idx"], want["right_idx"], f"{kind} right_idx")
    _eq(got["dist"], want["dist"], f"{kind} dist")
    assert got["n_matches"] == want["n_matches"], f"{kind} n_matches {got['n_matches']} vs {want['n_matches']}"
    m = want["right_idx"] >= 0
    if kind == "pinhole":
        _eq(got["sad"], want["sad"], "pinhole sad")
        assert np.all(np.abs(got["u_right"][m] - want["u_right"][m]) <= UR_TOL_PX), "u_right"
        assert np.all(np.abs(got["depth"][m] - want["depth"][m]) <= REL_TOL * np.abs(want["depth"][m])), "depth"
        assert np.all(got["u_right"][~m] == -1) and np.all(got["depth"][~m] == -1)
    else:
        d_ok = np.abs(got["depth"][m] - want["depth"][m]) <= REL_TOL * np.abs(want["depth"][m])
        assert np.all(d_ok), "fisheye depth"
        nrm = np.linalg.norm(want["xyz"][m], axis=1, keepdims=True)
        assert np.all(np.abs(got["xyz"][m] - want["xyz"][m]) <= REL_TOL * nrm), "fisheye xyz"
        assert np.all(got["depth"][~m] == -1) and np.all(got["xyz"][~m] == 0)


def compare_search(got, want, tag=""):
    for k in ("mp_match", "mp_dist", "kp_match"):
        _eq(got[k], want[k], f"search{tag} {k}")
    assert got["n_matches"] == want["n_matches"], f"search{tag} n_matches"


def compare_frame(got, want):
    if "stereo" in want:
        compare_stereo(want["kind"], got["stereo"], want["stereo"])
    assert len(got["search"]) == len(want["search"])
    for v, (g, w) in enumerate(zip(got["search"], want["search"])):
        compare_search(g, w, f"[{v}]")


def bit_equal(a, b):
    """Two device result dicts are identical to the last bit."""
    if "stereo" in a:
        for k, v in a["stereo"].items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v.view(np.uint8), b["stereo"][k].view(np.uint8)), k
            else:
                assert v == b["stereo"][k], k
    for g, w in zip(a["search"], b["search"]):
        for k, v in g.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, w[k]), k
            else:
                assert v == w[k], k
