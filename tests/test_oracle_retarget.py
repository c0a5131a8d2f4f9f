"""Pins of the oracle's whole retarget: k = 1 equals classic single-seam
carving written independently here (textbook DP, scipy Sobel), the first
iteration of every buffer equals the composition of the separately pinned
stages, and the invariants of Sec. 3.1 hold on the output (uniform width,
order of kept pixels, 8-connected disjoint seams, one mask per buffer)."""
import os

import numpy as np
import pytest
from scipy import ndimage

from paper_1903_03180_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sobel_energy(img):
    f = img.astype(np.int64)
    return np.abs(ndimage.sobel(f, axis=1, mode="nearest")) + np.abs(ndimage.sobel(f, axis=0, mode="nearest"))


def classic_seam_carve(img, n_remove):
    """Avidan-Shamir single-seam carving: recompute the gradient energy, run
    the cumulative DP (leftmost of equal predecessors), take the leftmost
    least last-row entry, trace it back, remove it; repeat."""
    img = img.copy()
    for _ in range(n_remove):
        H, W = img.shape
        e = sobel_energy(img)
        M = e.copy()
        back = np.zeros((H, W), dtype=np.int64)
        big = np.iinfo(np.int64).max // 4
        for i in range(1, H):
            prev = M[i - 1]
            left = np.concatenate(([big], prev[:-1]))
            right = np.concatenate((prev[1:], [big]))
            stack = np.stack([left, prev, right])
            arg = np.argmin(stack, axis=0)  # first (leftmost) minimum
            back[i] = np.arange(W) + arg - 1
            M[i] = e[i] + stack[arg, np.arange(W)]
        x = int(np.argmin(M[-1]))
        keep = np.ones((H, W), dtype=bool)
        for i in range(H - 1, -1, -1):
            keep[i, x] = False
            x = int(back[i, x])
        img = img[keep].reshape(H, W - 1)
    return img


@pytest.mark.parametrize("shape,remove", [((48, 64), 8), ((20, 31), 9), ((9, 6), 5), ((1, 7), 3), ((6, 1), 0)])
def test_k1_equals_classic_seam_carving(orc, shape, remove):
    H, W = shape
    rng = np.random.default_rng(H * W)
    img = synth.image_cfg1(3, H, W) if (H, W) == (48, 64) else rng.integers(0, 256, size=shape).astype(np.uint8)
    want = classic_seam_carve(img, remove)
    got = orc.retarget(img[None], W - remove, 1, mode=orc.GRADIENT, use_buffer=0)
    assert np.array_equal(got["out"][0], want)


def removed_carved_columns(mask_row, r):
    """Carved columns, at iteration r, of the pixels removed in iteration r."""
    alive = (mask_row == 0) | (mask_row > r)
    pos = np.cumsum(alive) - 1
    return pos[mask_row == r + 1]


def check_invariants(orc, frames, res, Wt):
    out, masks, bid, log = res["out"], res["masks"], res["buffer_id"], res["log"]
    N, H, W = masks.shape
    assert out.shape[2] == Wt
    # every row loses exactly W - Wt pixels
    assert np.all((masks > 0).sum(axis=2) == W - Wt)
    # kept pixels keep their order: output = input without masked pixels
    for t in range(N):
        keep = masks[t] == 0
        src = frames[t]
        want = src[keep].reshape((H, Wt) + src.shape[2:])
        assert np.array_equal(out[t], want)
    # all frames of a buffer share the mask
    for t in range(1, N):
        if bid[t] == bid[t - 1]:
            assert np.array_equal(masks[t], masks[t - 1])
    # per iteration: k_iter pixels per row, forming k_iter 8-connected seams
    for b in np.unique(bid):
        t = int(np.nonzero(bid == b)[0][0])
        rows = log[log[:, 0] == b]
        assert int(rows[:, 3].sum()) == W - Wt
        for r, (_, Wr, peff, kk) in enumerate(rows.tolist()):
            assert 1 <= kk <= min(peff, Wr - Wt)  # the caller's k caps it further
            cols = [removed_carved_columns(masks[t, i], r) for i in range(H)]
            assert all(len(c) == kk for c in cols)
            seams = np.stack(cols, axis=1)  # kk x H, sorted per row
            assert np.all(np.abs(np.diff(seams, axis=1)) <= 1)
            assert np.all(seams < Wr)


@pytest.mark.parametrize("seed,k,C", [(0, 3, 3), (1, 8, 1), (2, 1, 1), (3, 50, 3)])
def test_invariants_on_small_clips(orc, seed, k, C):
    clip = synth.make_clip(200 + seed, 12, 30, 52, C=C, n_obj=3, cut_at=6, lattice=8)
    Wt = 38
    res = orc.retarget(clip, Wt, k)
    check_invariants(orc, clip, res, Wt)
    for b in np.unique(res["buffer_id"]):
        rows = res["log"][res["log"][:, 0] == b]
        for _, Wr, peff, kk in rows.tolist():
            assert kk == min(k, peff, Wr - Wt)


def uniform_energy(orc, carved, T, ghost, mode):
    acc = 0
    for f in range(ghost, len(carved)):
        prev = carved[f - 1] if f > 0 else None
        acc = acc + orc.energy(carved[f], prev, mode).astype(np.int64)
    return (acc // T).astype(np.int32)


@pytest.mark.parametrize("mode", [1, 0])
def test_first_iteration_is_composition_of_stages(orc, mode):
    """Iteration 0 of every buffer: U = floor(mean energy) with the ghost as
    the first frame's predecessor, then DP, select, backtrack."""
    clip = synth.make_clip(31, 10, 22, 40, C=1, n_obj=3, cut_at=5, lattice=8)
    k, Wt = 4, 30
    res = orc.retarget(clip, Wt, k, mode=mode, anum=1, aden=5)
    bid = res["buffer_id"]
    for b in np.unique(bid):
        idx = np.nonzero(bid == b)[0]
        t0, T = int(idx[0]), len(idx)
        ghost = 1 if (mode == orc.MOTION and t0 > 0) else 0
        carved = [clip[t] for t in range(t0 - ghost, t0 + T)]
        U = uniform_energy(orc, carved, T, ghost, mode)
        ce, lab, d = orc.dp(U)
        ch, peff = orc.select(ce[-1], lab[-1], k, 40 - Wt)
        seams = orc.backtrack(d, ch)
        m = res["masks"][t0]
        for s in range(len(ch)):
            for i in range(22):
                assert m[i, seams[s, i]] == 1
        assert int((m == 1).sum()) == len(ch) * 22


def test_carried_motion_term_equals_carved_difference(orc):
    """Frames carved with the same seams: the difference of the carved frames
    is the original difference gathered through the column map, so the
    motion term can be carried with each pixel."""
    clip = synth.make_clip(41, 6, 18, 33, C=1, n_obj=2, lattice=8)
    res = orc.retarget(clip, 20, 5, mode=orc.MOTION, use_buffer=1, anum=1, aden=1)
    m = res["masks"]
    for t in range(1, 6):
        if res["buffer_id"][t] != res["buffer_id"][t - 1]:
            continue
        keep = m[t] == 0
        a = clip[t][keep].reshape(18, 20).astype(int)
        b = clip[t - 1][keep].reshape(18, 20).astype(int)
        D = np.abs(clip[t].astype(int) - clip[t - 1].astype(int))[keep].reshape(18, 20)
        assert np.array_equal(np.abs(a - b), D)


def test_single_frame_gradient_cfg1_shape(orc):
    img = synth.image_cfg1()
    res = orc.retarget(img[None], 56, 8, mode=orc.GRADIENT, use_buffer=0)
    check_invariants(orc, img[None], res, 56)


def test_degenerate_sizes(orc):
    one = np.array([[[5]]], dtype=np.uint8)
    res = orc.retarget(one, 1, 1)
    assert res["out"].tolist() == [[[5]]] and len(res["log"]) == 0
    row = np.arange(9, dtype=np.uint8).reshape(1, 1, 9)
    res = orc.retarget(row, 4, 2, mode=orc.GRADIENT, use_buffer=0)
    check_invariants(orc, row, res, 4)


def target_width(W, num, den):
    return (W * num) // den


def test_table1_target_width_rounding():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_target_widths.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 10
    for w, t, n, d in rows:
        assert target_width(int(w), int(n), int(d)) == int(t)


def test_height_retarget_is_width_retarget_of_the_transpose(orc):
    """Horizontal seams (Sec. 3.1, eq. 2): carving the height of a clip equals
    carving the width of its transpose; every output column keeps its
    pixels' order and loses exactly H - Ht of them."""
    from paper_1903_03180_amd import synth
    clip = synth.make_clip(41, 6, 30, 24, C=3, n_obj=2, lattice=8)
    r = orc.retarget_2d(clip, 24, 21, 4)
    assert r["out"].shape == (6, 21, 24, 3)
    m = r["masks"]
    assert np.all((m > 0).sum(axis=1) == 30 - 21)
    for t in range(6):
        for j in range(24):
            keep = m[t][:, j] == 0
            assert np.array_equal(r["out"][t][:, j], clip[t][keep, j])
    # 2-D: width first, then height of the result
    r2 = orc.retarget_2d(clip, 18, 21, 4)
    w = orc.retarget(clip, 18, 4)
    h = orc.retarget(np.swapaxes(w["out"], 1, 2), 21, 4)
    assert np.array_equal(r2["out"], np.swapaxes(h["out"], 1, 2))
    assert r2["masks"] is None and np.array_equal(r2["buffer_id"], w["buffer_id"])
