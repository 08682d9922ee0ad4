"""Index arithmetic the kernels rely on, restated on the host and checked
against brute force: the first output row of a pyramid level whose top tap
row reaches a given source row (closed form against bisection over the tap),
and the record deal of the batched search (segment ids written at their first
position of a round and a prefix maximum per 64 positions name every
position's segment and record, against laying all segments end to end)."""
import numpy as np


def _tap(x, n_in, n_out):
    """Top source row (or column) of output index x: floor(((2x + 1) n_in -
    n_out) / (2 n_out)), 0 below, clamped to n_in - 1."""
    num = (2 * x + 1) * n_in - n_out
    if num <= 0:
        return 0
    return min(num // (2 * n_out), n_in - 1)


def _first_row_bisect(Y, H, h):
    lo, hi = 0, h
    while lo < hi:
        mid = (lo + hi) // 2
        if _tap(mid, H, h) >= Y:
            hi = mid
        else:
            lo = mid + 1
    return lo


def _first_row_closed(Y, H, h):
    num = 2 * h * Y + h - H
    return 0 if num <= 0 else (num + 2 * H - 1) // (2 * H)


def test_pyramid_first_row_closed_form_matches_bisection():
    sizes = list(range(2, 90)) + [240, 333, 480, 512, 720, 1080]
    for H in sizes:
        levels = {max(1, int(round(H / 1.2 ** l))) for l in range(1, 8)} | {1, H}
        for h in sorted(levels):
            for Y in range(H):
                assert _first_row_closed(Y, H, h) == _first_row_bisect(Y, H, h), (Y, H, h)


def _deal(n, a, K=4):
    """The kernel's deal of one chunk: n[l, e] records of row e of lane l's
    window start at record a[l, e]; rounds of 64 * K positions, lane d taking
    positions d + 64 k.  Returns, per chunk position, (segment, record)."""
    R = n.shape[1]
    mine = n.sum(1)
    incl = np.cumsum(mine)
    total = int(incl[-1])
    st = (incl - mine)[:, None] + np.concatenate([np.zeros((64, 1), int), np.cumsum(n, 1)[:, :-1]], 1)
    delta = (a - st).reshape(-1)
    seg_of, rec_of = np.full(total, -1), np.full(total, -1)
    for g_lo in range(0, total, 64 * K):
        cnt = min(total - g_lo, 64 * K)
        mark = np.zeros(64 * K, int)
        for l in range(64):
            for e in range(R):
                A = st[l, e] - g_lo
                if n[l, e] > 0 and A < cnt and A + n[l, e] > 0:
                    assert mark[max(A, 0)] == 0, "two segments marked one position"
                    mark[max(A, 0)] = l * R + e + 1
        carry = 0
        for k in range(K):
            row = np.maximum(np.maximum.accumulate(mark[64 * k:64 * k + 64]), carry)
            carry = row[-1]
            for d in range(64):
                p = 64 * k + d
                if p < cnt:
                    s = row[d] - 1
                    seg_of[g_lo + p] = s
                    rec_of[g_lo + p] = g_lo + p + delta[s]
    return seg_of, rec_of


def test_striped_deal_names_every_record_once():
    rng = np.random.default_rng(11)
    for trial in range(120):
        kind = trial % 3
        if kind == 0:
            n = rng.integers(0, 5, (64, 4))
        elif kind == 1:
            n = np.where(rng.random((64, 4)) < 0.15, rng.integers(0, 200, (64, 4)), 0)
        else:
            n = np.zeros((64, 4), int)
            n[rng.integers(0, 64), rng.integers(0, 4)] = rng.integers(1, 900)
        a = rng.integers(0, 60000, (64, 4))
        seg_of, rec_of = _deal(n, a)
        want_seg = [l * 4 + e for l in range(64) for e in range(4) for _ in range(n[l, e])]
        want_rec = [a[l, e] + i for l in range(64) for e in range(4) for i in range(n[l, e])]
        assert seg_of.tolist() == want_seg
        assert rec_of.tolist() == want_rec


def _bins_walk(ranges, G=4, U=2):
    """The pinhole scan's positions over (start, count) ranges of up to three
    level bins: lane `sub` of G reads positions sub + G u + U G k, clamped to
    total - 1; returns the records the in-range positions name and every
    record a clamped read touches."""
    (s0, n0), (s1, n1), (s2, n2) = (list(ranges) + [(0, 0)] * 3)[:3]
    n01, total = n0 + n1, n0 + n1 + n2

    def at(p):
        p = min(p, total - 1)
        return s0 + p if p < n0 else s1 + (p - n0) if p < n01 else s2 + (p - n01)

    named, touched = {}, set()
    for sub in range(G):
        if total == 0:
            continue
        for u in range(U):
            touched.add(at(sub + u * G))
        p0 = sub
        while p0 < total:
            for u in range(U):
                p = p0 + u * G
                if p < total:
                    named[p] = at(p)
                touched.add(at(p0 + (U + u) * G))
            p0 += U * G
    return [named[p] for p in sorted(named)], touched


def test_bins_walk_names_every_record_once_in_order():
    rng = np.random.default_rng(5)
    for trial in range(400):
        k = 1 + trial % 3
        counts = rng.integers(0, 40, k)
        if trial % 7 == 0:
            counts[rng.integers(0, k)] = 0
        starts = np.cumsum(rng.integers(0, 500, k)) + np.concatenate([[0], np.cumsum(counts)[:-1]])
        ranges = [(int(a), int(n)) for a, n in zip(starts, counts)]
        want = [a + i for a, n in ranges for i in range(n)]
        got, touched = _bins_walk(ranges, G=int(rng.choice([1, 2, 4, 8, 16])))
        assert got == want, (ranges, got[:10])
        assert touched <= set(want), (ranges, sorted(touched - set(want))[:5])
