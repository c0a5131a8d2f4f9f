"""Pins of the oracle's buffer test (Sec. 3.2, eqs. 7-9): the integer square
root against Python's math.isqrt, exact cases of the discretised ASDE, the
worst-case buffer that eq. (9) models (Fig. 4, at two resolutions), and the
decision against eq. (9) evaluated as printed with 60-digit decimals."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

getcontext().prec = 60


def test_isqrt_against_math_isqrt(orc):
    rng = np.random.default_rng(1)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**52 - 1, 2**52, 2**53 + 1, 2**62, 2**64 - 1]
    for r in [3, 2**20 + 7, 2**31 - 1, 2**32 - 1]:
        vals += [r * r - 1, r * r, r * r + 1]
    vals += [int(x) for x in rng.integers(0, 2**63, size=2000, dtype=np.uint64)]
    for v in vals:
        v = min(v, 2**64 - 1)
        assert orc.isqrt(v) == math.isqrt(v), v


def moments(es):
    es = [e.astype(np.uint64) for e in es]
    return sum(es), sum(e * e for e in es)


def test_two_frames_exact(orc):
    # n = 2: 2 (a^2 + b^2) - (a + b)^2 = (a - b)^2, so S = sum |a - b| exactly
    rng = np.random.default_rng(2)
    a = rng.integers(0, 7651, size=(31, 47))
    b = rng.integers(0, 7651, size=(31, 47))
    s1, s2 = moments([a, b])
    assert orc.asde_sum(s1, s2, 2) == int(np.abs(a - b).sum())


def test_identical_frames_zero(orc):
    a = np.random.default_rng(3).integers(0, 7651, size=(20, 20))
    for n in (1, 2, 5, 40):
        s1, s2 = moments([a] * n)
        S = orc.asde_sum(s1, s2, n)
        assert S == 0
        assert not orc.reject(S, n, a.size, 7650, 1, 5)


def test_against_numpy_population_std(orc):
    # floor per pixel makes S at most one unit per pixel below n * sum(std)
    rng = np.random.default_rng(4)
    for n in (2, 3, 7, 16):
        es = [rng.integers(0, 7651, size=(25, 19)) for _ in range(n)]
        s1, s2 = moments(es)
        S = orc.asde_sum(s1, s2, n)
        ref = n * np.std(np.stack(es).astype(np.float64), axis=0).sum()
        assert ref - es[0].size - 1e-6 <= S <= ref + 1e-6


def phi_eq9(n, alpha, maxval):
    """Eq. (9) exactly as printed, in 60-digit decimals."""
    n = Decimal(n)
    m = Decimal(maxval)
    inner = ((m - m / n) ** 2 + (n - 1) * (m / n) ** 2) / n
    return Decimal(alpha) * inner.sqrt()


@pytest.mark.parametrize("H,W", [(480, 640), (720, 1280)])
def test_worst_case_buffer_resolution_independent(orc, H, W):
    """n-1 frames at the lowest energy and one at the highest, at every pixel:
    the buffer eq. (9) models.  ASDE then equals phi(n) / alpha at any
    resolution (Fig. 4); with n - 1 a perfect square the discretised sum is
    exact, so alpha = 1 is the boundary that must not reject and any alpha
    below it must reject."""
    E = 7650
    for m in (1, 2, 3):
        n = m * m + 1
        s1 = np.full(H * W, E, dtype=np.uint64)
        s2 = np.full(H * W, E * E, dtype=np.uint64)
        S = orc.asde_sum(s1, s2, n)
        assert S == H * W * E * m
        asde = Decimal(S) / (Decimal(n) * H * W)
        assert abs(asde - phi_eq9(n, 1, E)) < Decimal("1e-40")
        assert not orc.reject(S, n, H * W, E, 1, 1)
        assert orc.reject(S, n, H * W, E, 99, 100)


def test_threshold_closed_form_small_n():
    for n in range(1, 8):
        for alpha in ("0.15", "0.2", "0.25"):
            closed = Decimal(alpha) * 7650 * Decimal(n - 1).sqrt() / n
            assert abs(phi_eq9(n, Decimal(alpha), 7650) - closed) < Decimal("1e-50")


def test_reject_matches_eq9_decimal(orc):
    rng = np.random.default_rng(6)
    checked = 0
    for _ in range(4000):
        n = int(rng.integers(2, 400))  # a candidate buffer holds at least two frames
        H, W = int(rng.integers(1, 3000)), int(rng.integers(1, 3000))
        emax = int(rng.choice([1530, 7650]))
        anum, aden = int(rng.integers(0, 30)), int(rng.integers(1, 40))
        phi = phi_eq9(n, Decimal(anum) / Decimal(aden), emax)
        target = phi * n * H * W  # S at which ASDE = phi
        S = max(0, int(target) + int(rng.integers(-3, 4)))
        asde = Decimal(S) / (Decimal(n) * H * W)
        if abs(asde - phi) < Decimal("1e-30"):
            continue  # exact ties are decided by the strict inequality below
        want = asde > phi
        assert orc.reject(S, n, H * W, emax, anum, aden) == want, (S, n, H, W, emax, anum, aden)
        checked += 1
    assert checked > 3000


def test_reject_never_at_n1(orc):
    assert not orc.reject(10**12, 1, 4, 7650, 1, 5)
    assert not orc.reject(10**12, 1, 4, 7650, 0, 5)


def _float_segment(Y, anum, aden, mode, orc):
    """Segmentation from eqs. (7)-(9) in floating point (numpy std, printed
    phi), returning decisions and the margin of each test."""
    N = Y.shape[0]
    E = [orc.energy(Y[t], Y[t - 1] if t else None, mode).astype(np.float64) for t in range(N)]
    emax = orc.energy_max(mode)
    bid = [0]
    buf = [E[0]]
    margins = [None]
    for t in range(1, N):
        cand = buf + [E[t]]
        n = len(cand)
        asde = float(np.std(np.stack(cand), axis=0).mean())
        phi = float(phi_eq9(n, Decimal(anum) / Decimal(aden), emax))
        margins.append(asde - phi)
        if asde > phi:
            bid.append(bid[-1] + 1)
            buf = [E[t]]
        else:
            bid.append(bid[-1])
            buf = cand
    return np.array(bid), margins


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_segmentation_matches_float_reading(orc, seed):
    from paper_1903_03180_amd import synth
    clip = synth.make_clip(100 + seed, 14, 24, 40, C=1, n_obj=3, max_speed=5, cut_at=7, lattice=8)
    for anum, aden in ((3, 20), (1, 5), (1, 4), (1, 40)):
        bid, st = orc.segment(clip, orc.MOTION, 1, anum, aden)
        fb, margins = _float_segment(clip, anum, aden, orc.MOTION, orc)
        # discretisation moves ASDE by less than 1/n; decisions must agree
        # wherever the float margin is wider than that
        for t in range(1, len(bid)):
            n_here = int(np.sum(fb[:t] == fb[t - 1])) + 1
            if abs(margins[t]) > 1.0 / n_here + 1e-9:
                assert (bid[t] != bid[t - 1]) == (fb[t] != fb[t - 1]), (t, margins[t])
            else:
                break  # later decisions depend on this borderline one


def test_static_clip_is_one_buffer(orc):
    from paper_1903_03180_amd import synth
    fr = synth.make_clip(5, 1, 20, 30, C=1, n_obj=2)[0]
    clip = np.stack([fr] * 9)
    bid, st = orc.segment(clip, orc.MOTION, 1, 1, 5)
    assert bid.tolist() == [0] * 9


def test_hard_cut_breaks_and_trigger_starts_next_buffer(orc):
    rng = np.random.default_rng(8)
    a = np.zeros((16, 16), dtype=np.uint8)
    b = rng.integers(0, 2, size=(16, 16)).astype(np.uint8) * 255
    clip = np.stack([a] * 4 + [b] * 4)
    bid, st = orc.segment(clip, orc.MOTION, 1, 1, 5)
    assert bid[:4].tolist() == [0] * 4
    assert bid[4] == 1


def test_max_buffer_and_no_buffer(orc):
    fr = np.full((5, 7), 9, dtype=np.uint8)
    clip = np.stack([fr] * 7)
    bid, _ = orc.segment(clip, orc.MOTION, 1, 1, 5, max_buffer=3)
    assert bid.tolist() == [0, 0, 0, 1, 1, 1, 2]
    bid, _ = orc.segment(clip, orc.MOTION, 0, 1, 5)
    assert bid.tolist() == list(range(7))
