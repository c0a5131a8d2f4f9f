"""Pins of the oracle's seam-memorisation mode (Sec. 5 names seam
memorisation as future work; the reading: with period m >= 2 only buffers
b with b mod m == 0 are carved, and every other buffer removes from each of
its frames the pixels that buffer b - (b mod m) removed).

The pins do not go through the oracle's own memorisation code path to
derive what it should produce: carved buffers must equal the ordinary
retarget, a memorised frame's output must be its input row filtered by the
source buffer's mask (numpy boolean indexing), and on a static clip, where
every buffer would pick the same seams, memorisation must change nothing."""
import numpy as np
import pytest

from paper_1903_03180_amd import synth


def spans(bid):
    """(t0, T) of each buffer from per-frame buffer ids."""
    out, t0 = [], 0
    for t in range(1, len(bid) + 1):
        if t == len(bid) or bid[t] != bid[t - 1]:
            out.append((t0, t - t0))
            t0 = t
    return out


def filter_rows(frame, mask):
    """Each row of `frame` without the pixels whose mask entry is nonzero."""
    return np.stack([frame[i][mask[i] == 0] for i in range(frame.shape[0])])


@pytest.mark.parametrize("m", [0, 1])
def test_period_one_is_plain(orc, m):
    clip = synth.make_clip(41, 12, 24, 60, C=3, n_obj=3, cut_at=6, lattice=8)
    a = orc.retarget(clip, 44, 4, max_buffer=3)
    b = orc.retarget(clip, 44, 4, max_buffer=3, memo_period=m)
    for key in ("out", "masks", "buffer_id", "log"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("m,C,k", [(2, 3, 4), (3, 1, 6), (4, 3, 1000)])
def test_memorised_buffers(orc, m, C, k):
    N, H, W, Wt = 20, 26, 64, 45
    clip = synth.make_clip(42 + m, N, H, W, C=C, n_obj=4, max_speed=5, lattice=8)
    plain = orc.retarget(clip, Wt, k, max_buffer=2)
    memo = orc.retarget(clip, Wt, k, max_buffer=2, memo_period=m)
    bid = plain["buffer_id"]
    assert np.array_equal(memo["buffer_id"], bid)  # segmentation unchanged
    bufs = spans(bid)
    assert len(bufs) >= 2 * m
    differs = False
    for b, (t0, T) in enumerate(bufs):
        sl = slice(t0, t0 + T)
        if b % m == 0:
            # carved buffers: exactly the ordinary result
            assert np.array_equal(memo["out"][sl], plain["out"][sl])
            assert np.array_equal(memo["masks"][sl], plain["masks"][sl])
            continue
        s0 = bufs[b - b % m][0]
        src_mask = plain["masks"][s0]
        differs |= not np.array_equal(plain["masks"][t0], src_mask)
        for f in range(t0, t0 + T):
            assert np.array_equal(memo["masks"][f], src_mask)
            assert np.array_equal(memo["out"][f], filter_rows(clip[f], src_mask))
    # the moving clip makes at least one memorised buffer's own seams differ,
    # so the checks above distinguish reuse from carving
    assert differs
    # the record holds the carved buffers' iterations only, as in the plain run
    keep = np.isin(plain["log"][:, 0], [b for b in range(len(bufs)) if b % m == 0])
    assert np.array_equal(memo["log"], plain["log"][keep])


@pytest.mark.parametrize("mode", [0, 1])
def test_static_clip_memorisation_changes_nothing(orc, mode):
    """Identical frames in buffers forced to 3 frames: every buffer has the
    same uniform energy (the motion term is zero, the first frame's included),
    hence the same seams, so the memorised run equals the plain one."""
    frame = synth.make_clip(47, 1, 30, 70, C=3, n_obj=3, lattice=8)[0]
    clip = np.repeat(frame[None], 13, axis=0)
    plain = orc.retarget(clip, 52, 5, mode=mode, max_buffer=3)
    assert len(spans(plain["buffer_id"])) == 5
    for m in (2, 3, 5):
        memo = orc.retarget(clip, 52, 5, mode=mode, max_buffer=3, memo_period=m)
        assert np.array_equal(memo["out"], plain["out"])
        assert np.array_equal(memo["masks"], plain["masks"])


def test_memorisation_in_2d(orc):
    """Both passes follow the rule: the width pass's memorised frames are
    filtered by their source's removal before the height pass."""
    clip = synth.make_clip(48, 10, 36, 40, C=1, n_obj=3, lattice=8)
    a = orc.retarget_2d(clip, 30, 28, 4, max_buffer=2, memo_period=2)
    w = orc.retarget(clip, 30, 4, max_buffer=2, memo_period=2)
    h = orc.retarget(np.ascontiguousarray(np.swapaxes(w["out"], 1, 2)), 28, 4, max_buffer=2, memo_period=2)
    assert np.array_equal(a["out"], np.swapaxes(h["out"], 1, 2))
