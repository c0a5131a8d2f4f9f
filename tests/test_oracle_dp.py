"""Pins of the oracle's cumulative-energy DP (eq. 4), parent labels (Sec. 3.1,
eq. 5), per-parent least child and top-k (eq. 6) and backtracking, by brute
force: every 8-connected seam (eq. 1) of a tiny image is enumerated and
costed (eq. 3) without any dynamic programme."""
import itertools

import numpy as np
import pytest


def enumerate_paths(u, rows):
    """All 8-connected paths through rows 0..rows-1: (cost, cols tuple)."""
    H, W = u.shape
    out = []
    for x0 in range(W):
        for moves in itertools.product((-1, 0, 1), repeat=rows - 1):
            cols = [x0]
            ok = True
            for m in moves:
                x = cols[-1] + m
                if x < 0 or x >= W:
                    ok = False
                    break
                cols.append(x)
            if ok:
                out.append((sum(int(u[i, c]) for i, c in enumerate(cols)), tuple(cols)))
    return out


def canonical(paths):
    """Per end pixel: least cost, and among least-cost paths the one that is
    lexicographically smallest read from the bottom up, x(i-1), x(i-2), ...,
    x(0) (what leftmost backtracking returns)."""
    best = {}
    for cost, cols in paths:
        end = cols[-1]
        key = (cost, tuple(reversed(cols[:-1])))
        if end not in best or key < best[end][0]:
            best[end] = (key, cols)
    return {end: (k[0], cols) for end, (k, cols) in best.items()}


def brute(u):
    H, W = u.shape
    ce = np.zeros((H, W), dtype=np.int64)
    lab = np.zeros((H, W), dtype=np.int64)
    d = np.zeros((H, W), dtype=np.int64)
    seam_of = {}
    for i in range(H):
        can = canonical(enumerate_paths(u, i + 1))
        for j in range(W):
            cost, cols = can[j]
            ce[i, j] = cost
            lab[i, j] = cols[0]
            d[i, j] = cols[-2] - j if i > 0 else 0
            if i == H - 1:
                seam_of[j] = cols
    return ce, lab, d, seam_of


def brute_select(ce_last, lab_last, k, limit):
    per_parent = {}
    for j, (c, l) in enumerate(zip(ce_last.tolist(), lab_last.tolist())):
        if l not in per_parent or c < per_parent[l][0]:
            per_parent[l] = (c, j)
    ranked = sorted(per_parent.values())
    kk = min(k, len(ranked), limit)
    return sorted(j for _, j in ranked[:kk]), len(per_parent)


CASES = [(1, 1), (1, 4), (4, 1), (2, 2), (3, 2), (2, 5), (5, 6), (6, 7), (7, 8), (8, 6)]


@pytest.mark.parametrize("H,W", CASES)
@pytest.mark.parametrize("hi", [1, 3, 40])
def test_dp_labels_dirs_against_brute_force(orc, H, W, hi):
    rng = np.random.default_rng(H * 100 + W * 10 + hi)
    for trial in range(3 if H * W > 30 else 6):
        u = rng.integers(0, hi + 1, size=(H, W)).astype(np.int32)
        ce, lab, d = orc.dp(u)
        bce, blab, bd, _ = brute(u)
        assert np.array_equal(ce, bce)
        assert np.array_equal(lab, blab)
        assert np.array_equal(d, bd)


@pytest.mark.parametrize("H,W", CASES)
@pytest.mark.parametrize("k", [1, 2, 3, 8])
def test_select_and_backtrack_against_brute_force(orc, H, W, k):
    rng = np.random.default_rng(H * 1000 + W * 10 + k)
    for trial in range(4):
        u = rng.integers(0, 4, size=(H, W)).astype(np.int32)
        ce, lab, d = orc.dp(u)
        bce, blab, bd, seam_of = brute(u)
        for limit in (W, max(W - 2, 0), 1):
            ch, peff = orc.select(ce[-1], lab[-1], k, limit)
            bch, bpeff = brute_select(bce[-1], blab[-1], k, limit)
            assert peff == bpeff
            assert ch.tolist() == bch
            seams = orc.backtrack(d, ch)
            for s, c in enumerate(ch.tolist()):
                assert tuple(seams[s].tolist()) == seam_of[c]
                # each traced seam ends at its own parent label
                assert seams[s][0] == lab[-1][c]


def test_select_fewer_parents_than_k(orc):
    # a single deep valley: every child descends from one parent
    H, W = 5, 6
    u = np.full((H, W), 9, dtype=np.int32)
    u[0, 2] = 0
    u[1:, :] = 0
    ce, lab, d = orc.dp(u)
    ch, peff = orc.select(ce[-1], lab[-1], 4, W)
    assert peff == len(set(lab[-1].tolist()))
    assert len(ch) == min(4, peff)


@pytest.mark.parametrize("seed", range(6))
def test_labels_monotone_and_seams_disjoint(orc, seed):
    """Under the leftmost tie-break the predecessor map is non-decreasing in
    the column, so labels never decrease along a row, and seams of different
    children never share a pixel; they keep their order in every row."""
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(2, 60)), int(rng.integers(2, 90))
    u = rng.integers(0, int(rng.choice([2, 5, 1000])), size=(H, W)).astype(np.int32)
    ce, lab, d = orc.dp(u)
    assert np.all(np.diff(lab, axis=1) >= 0)
    pred = np.arange(W)[None, :] + d
    assert np.all(np.diff(pred[1:], axis=1) >= 0)
    assert d.min() >= -1 and d.max() <= 1
    assert pred.min() >= 0 and pred.max() < W
    ch, peff = orc.select(ce[-1], lab[-1], W, W)
    assert peff == len(set(lab[-1].tolist()))
    seams = orc.backtrack(d, ch)
    if len(ch) > 1:
        assert np.all(np.diff(seams, axis=0) > 0)
    assert np.all(np.abs(np.diff(seams, axis=1)) <= 1)
    assert np.array_equal(seams[:, 0], lab[-1][ch])
