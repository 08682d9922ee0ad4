"""Pins of the oracle's local-map maintenance (Update Local Map's output set
kept in device memory, where the search reads it).

Each record carries a unique tag (its dmin), so the expected layout follows
from properties of the rule rather than from a second copy of it: the new map
holds exactly the surviving and inserted records; survivors below the new
count keep their slots; the removed slots below it take the surviving tail
points in ascending order; inserted points follow in order; invalid lists and
capacity overflows leave the map untouched.
"""
import numpy as np
import pytest

import oracle


def _map(n, seed):
    rng = np.random.default_rng(seed)
    return {"pos": rng.normal(0, 5, (n, 3)).astype(np.float32),
            "normal": rng.normal(0, 1, (n, 3)).astype(np.float32),
            "dmin": np.arange(n, dtype=np.float32),                      # tag
            "dmax": rng.uniform(1, 20, n).astype(np.float32),
            "desc": rng.integers(0, 256, (n, 32), dtype=np.uint8)}


def _records(mp):
    return {float(mp["dmin"][i]): (mp["pos"][i].tobytes() + mp["normal"][i].tobytes() +
                                   mp["dmax"][i].tobytes() + mp["desc"][i].tobytes())
            for i in range(len(mp["dmin"]))}


def _check(old, remove, ins, new, capacity):
    n, m, r = len(old["dmin"]), len(ins["dmin"]), len(remove)
    n1 = n - r
    assert len(new["dmin"]) == n1 + m <= capacity
    # exactly the surviving and inserted records, each once
    want = _records(old)
    for i in remove:
        del want[float(old["dmin"][i])]
    want.update(_records(ins))
    got = _records(new)
    assert len(got) == len(new["dmin"]) and got == want
    gone = set(int(i) for i in remove)
    # survivors below n1 keep their slots
    for i in range(n1):
        if i not in gone:
            assert new["dmin"][i] == old["dmin"][i]
    # holes take the tail survivors in ascending order
    holes = [i for i in range(n1) if i in gone]
    tail = [i for i in range(n1, n) if i not in gone]
    assert len(holes) == len(tail)
    for h, t in zip(holes, tail):
        assert new["dmin"][h] == old["dmin"][t]
    # inserted points in order after n1
    assert np.array_equal(new["dmin"][n1:], ins["dmin"])


CASES = [
    ("nothing", 50, [], 0),
    ("insert only", 50, [], 7),
    ("head", 50, [0, 1, 2, 10], 0),
    ("tail only", 50, [49, 48, 45], 3),
    ("mixed", 200, [5, 199, 100, 17, 150, 160, 3, 120], 12),
    ("everything", 30, list(range(30)), 4),
    ("all but one", 30, list(range(1, 30)), 0),
    ("empty map", 0, [], 5),
]


@pytest.mark.parametrize("name,n,remove,m", CASES)
def test_map_update_rule(name, n, remove, m):
    old = _map(n, 1)
    ins = _map(m, 2)
    ins["dmin"] += 100000.0
    cap = n + m + 3
    new = oracle.map_update(old, cap, remove, ins)
    assert new is not None
    _check(old, remove, ins, new, cap)


def test_random_edit_sequences():
    rng = np.random.default_rng(3)
    mp = _map(500, 4)
    tag = 100000.0
    cap = 800
    for step in range(30):
        n = len(mp["dmin"])
        r = rng.choice(n, rng.integers(0, min(n, 60) + 1), replace=False)
        m = int(rng.integers(0, 60))
        ins = _map(m, 100 + step)
        ins["dmin"] = (tag + np.arange(m)).astype(np.float32)
        tag += m
        if n - len(r) + m > cap:
            m = 0
            ins = {k: v[:0] for k, v in ins.items()}
        new = oracle.map_update(mp, cap, r, ins)
        _check(mp, r, ins, new, cap)
        mp = new


@pytest.mark.parametrize("remove,m,cap", [([3, 3], 0, 100), ([50], 0, 100), ([-1], 0, 100),
                                          ([], 11, 60), ([1, 2], 13, 60)])
def test_invalid_edits_are_rejected(remove, m, cap):
    old = _map(50, 5)
    ins = _map(m, 6)
    assert oracle.map_update(old, cap, remove, ins) is None


def test_exact_capacity_is_accepted():
    old = _map(40, 7)
    ins = _map(5, 8)
    ins["dmin"] += 1000.0
    new = oracle.map_update(old, 43, [0, 39], ins)
    assert new is not None and len(new["dmin"]) == 43
