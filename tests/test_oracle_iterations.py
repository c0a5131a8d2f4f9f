"""Pin of the oracle's later iterations (r >= 1) of every buffer.

For every iteration r of every buffer the test rebuilds, with numpy only,
the buffer's frames as they stand after iterations 0..r-1: each original
frame filtered by the buffer's mask (pixels with mask 0 or mask > r are
still present).  The predecessor of the buffer's first frame (the ghost,
motion energy only) is the original frame before the buffer filtered by the
same mask.  From these frames it recomputes the uniform energy of Sec. 3.2
(floor of the mean of the frames' energies) with its own Sobel energy
(scipy) and the motion term of Sec. 3.3 (e = 2 G + 18 |Y_t - Y_{t-1}|), runs
the brute-force-pinned DP, selection and backtrack stages of eqs. (4)-(6),
and requires that the seams it finds are exactly the pixels the oracle
marked r + 1, and that the oracle's log row (W_r, P_eff, k_iter) matches.

A mistake in how the oracle carves the predecessor or the ghost, averages
the energies, or moves the iteration on would change some iteration's seams
or log row and fail here.
"""
import numpy as np
import pytest
from scipy import ndimage

from paper_1903_03180_amd import synth


def sobel_l1(img):
    f = img.astype(np.int64)
    return np.abs(ndimage.sobel(f, axis=1, mode="nearest")) + np.abs(ndimage.sobel(f, axis=0, mode="nearest"))


def energy_np(y, yprev, motion):
    """Sec. 3.3 with the gradient and difference maps brought to a common
    range: 2 G + 18 |dY| (motion), G (gradient); no term without a
    predecessor."""
    g = sobel_l1(y)
    if not motion:
        return g
    e = 2 * g
    if yprev is not None:
        e = e + 18 * np.abs(y.astype(np.int64) - yprev.astype(np.int64))
    return e


def carve(frame, mask, r):
    """The frame after iterations 0..r-1 of its buffer: the pixels whose
    removal iteration is r or later (mask > r) or never (mask == 0)."""
    H = frame.shape[0]
    alive = (mask == 0) | (mask > r)
    return frame[alive].reshape((H, -1) + frame.shape[2:])


def check_every_iteration(orc, luma, res, k, Wt, motion, ghost="carved"):
    masks, bid, log = res["masks"], res["buffer_id"], res["log"]
    N, H, W = luma.shape
    n_checked = 0
    for b in np.unique(bid):
        idx = np.nonzero(bid == b)[0]
        t0, T = int(idx[0]), len(idx)
        m = masks[t0]
        rows = log[log[:, 0] == b]
        has_ghost = motion and t0 > 0
        Wr = W
        for r, (_, lWr, lpeff, lkk) in enumerate(rows.tolist()):
            assert lWr == Wr
            frames = [carve(luma[t], m, r) for t in range(t0, t0 + T)]
            prev0 = None
            if has_ghost and ghost == "carved":
                prev0 = carve(luma[t0 - 1], m, r)
            elif has_ghost and ghost == "cropped":  # a wrong reading, for the sensitivity test
                prev0 = luma[t0 - 1][:, :Wr]
            acc = np.zeros((H, Wr), dtype=np.int64)
            for f in range(T):
                prev = frames[f - 1] if f > 0 else prev0
                acc += energy_np(frames[f], prev, motion)
            U = (acc // T).astype(np.int32)
            ce, lab, d = orc.dp(U)
            ch, peff = orc.select(ce[-1], lab[-1], k, Wr - Wt)
            seams = orc.backtrack(d, ch)
            assert (peff, len(ch)) == (lpeff, lkk), (b, r)
            # the pixels removed in iteration r, in carved columns of iteration r
            alive = (m == 0) | (m > r)
            pos = np.cumsum(alive, axis=1) - 1
            for i in range(H):
                got = pos[i][m[i] == r + 1]
                assert np.array_equal(np.sort(seams[:, i]), got), (b, r, i)
            Wr -= lkk
            n_checked += 1
        assert Wr == Wt
    return n_checked


@pytest.mark.parametrize("seed,N,H,W,Wt,k,cut", [
    (51, 10, 22, 40, 27, 3, 5),    # cut mid-clip: a ghost-led buffer
    (52, 12, 18, 33, 20, 5, 4),
    (53, 9, 14, 29, 12, 2, 6),     # many iterations per buffer
    (54, 8, 11, 24, 9, 16, 3),     # k above the number of parents
])
def test_motion_every_iteration_recomputed(orc, seed, N, H, W, Wt, k, cut):
    clip = synth.make_clip(seed, N, H, W, C=1, n_obj=3, cut_at=cut, lattice=8)
    res = orc.retarget(clip, Wt, k, mode=orc.MOTION, anum=1, aden=5)
    assert len(np.unique(res["buffer_id"])) >= 2  # the cut opens a ghost-led buffer
    n = check_every_iteration(orc, clip, res, k, Wt, motion=True)
    assert n >= 2 * len(np.unique(res["buffer_id"]))


def test_motion_every_iteration_rgb(orc):
    """RGB: the energy is that of the luma (pinned separately), the same
    seams are removed from the colour frames."""
    clip = synth.make_clip(55, 8, 16, 30, C=3, n_obj=2, cut_at=4, lattice=8)
    res = orc.retarget(clip, 21, 3, mode=orc.MOTION)
    luma = orc.luma(clip)
    check_every_iteration(orc, luma, res, 3, 21, motion=True)


def test_motion_every_iteration_capped_buffers(orc):
    """max_buffer cuts buffers with no scene change, so every later buffer
    has a ghost whose pixels move in step with the buffer's frames."""
    clip = synth.make_clip(56, 9, 15, 28, C=1, n_obj=3, lattice=8)
    res = orc.retarget(clip, 19, 4, mode=orc.MOTION, max_buffer=3)
    assert len(np.unique(res["buffer_id"])) == 3
    check_every_iteration(orc, clip, res, 4, 19, motion=True)


def test_gradient_every_iteration(orc):
    clip = synth.make_clip(57, 7, 13, 26, C=1, n_obj=2, cut_at=3, lattice=8)
    res = orc.retarget(clip, 15, 3, mode=orc.GRADIENT, anum=1, aden=5)
    check_every_iteration(orc, clip, res, 3, 15, motion=False)


@pytest.mark.parametrize("wrong", ["none", "cropped"])
def test_check_rejects_other_ghost_readings(orc, wrong):
    """The check tells the carved ghost from two plausible mistakes: no
    predecessor for a buffer's first frame, or the original frame before
    the buffer cut to the current width instead of carved with the
    buffer's seams.  Checking the oracle's run under either of them fails."""
    clip = synth.make_clip(51, 10, 22, 40, C=1, n_obj=3, cut_at=5, lattice=8)
    res = orc.retarget(clip, 27, 3, mode=orc.MOTION)
    check_every_iteration(orc, clip, res, 3, 27, motion=True)
    with pytest.raises(AssertionError):
        check_every_iteration(orc, clip, res, 3, 27, motion=True, ghost=wrong)
