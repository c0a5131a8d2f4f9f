"""Pins of the oracle's luma and energy (Sec. 3.3) to facts fixed outside it:
closed forms of the Sobel operator, scipy's Sobel filter, and the maximum of
the energy found by enumerating the vertices of the pixel box."""
import itertools

import numpy as np
import pytest
from scipy import ndimage


def test_luma_special_values(orc):
    rgb = np.array([[255, 255, 255], [0, 0, 0], [255, 0, 0], [0, 255, 0], [0, 0, 255]], dtype=np.uint8)
    assert orc.luma(rgb).tolist() == [255, 0, 77, 149, 29]


def test_luma_grey_is_identity(orc):
    v = np.arange(256, dtype=np.uint8)
    rgb = np.stack([v, v, v], axis=-1)
    assert np.array_equal(orc.luma(rgb), v)


def test_luma_monotone_in_each_channel(orc):
    rng = np.random.default_rng(0)
    base = rng.integers(0, 255, size=(1000, 3)).astype(np.uint8)
    y0 = orc.luma(base).astype(int)
    for c in range(3):
        b2 = base.copy()
        b2[:, c] += 1
        assert np.all(orc.luma(b2).astype(int) >= y0)


def test_constant_image_has_zero_gradient(orc):
    y = np.full((7, 9), 123, dtype=np.uint8)
    assert not orc.energy(y).any()


@pytest.mark.parametrize("c,a,b", [(1, 10, 250), (4, 200, 3), (8, 0, 255)])
def test_vertical_step(orc, c, a, b):
    H, W = 6, 9
    y = np.full((H, W), a, dtype=np.uint8)
    y[:, c:] = b
    e = orc.energy(y)
    want = np.zeros((H, W), dtype=np.int32)
    want[:, c - 1] = 4 * abs(b - a)
    want[:, c] = 4 * abs(b - a)
    assert np.array_equal(e, want)


def test_horizontal_ramp(orc):
    s = 3
    H, W = 5, 12
    y = np.tile((np.arange(W) * s).astype(np.uint8), (H, 1))
    e = orc.energy(y)
    assert np.all(e[:, 1:-1] == 8 * s)
    assert np.all(e[:, 0] == 4 * s) and np.all(e[:, -1] == 4 * s)


def test_single_column_and_single_pixel(orc):
    y = (np.arange(6) * 7).astype(np.uint8).reshape(6, 1)
    e = orc.energy(y)
    # W = 1: both side columns are the column itself, so Gx = 0 and
    # Gy = 4 (y[i+1] - y[i-1]) with replicated rows.
    want = [4 * abs(int(y[min(i + 1, 5), 0]) - int(y[max(i - 1, 0), 0])) for i in range(6)]
    assert e[:, 0].tolist() == want
    assert orc.energy(np.array([[77]], dtype=np.uint8)).tolist() == [[0]]


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (5, 1), (2, 2), (17, 23), (64, 48), (3, 130)])
def test_matches_scipy_sobel(orc, shape):
    rng = np.random.default_rng(sum(shape))
    y = rng.integers(0, 256, size=shape).astype(np.uint8)
    f = y.astype(np.int64)
    gx = ndimage.sobel(f, axis=1, mode="nearest")
    gy = ndimage.sobel(f, axis=0, mode="nearest")
    assert np.array_equal(orc.energy(y), (np.abs(gx) + np.abs(gy)).astype(np.int32))


def test_motion_term(orc):
    rng = np.random.default_rng(5)
    y = rng.integers(0, 200, size=(13, 17)).astype(np.uint8)
    g = orc.energy(y)
    # identical frames: difference term vanishes
    assert np.array_equal(orc.energy(y, y, orc.MOTION), 2 * g)
    # frame plus a constant c: difference term is 18 c everywhere
    y2 = (y + 37).astype(np.uint8)
    assert np.array_equal(orc.energy(y2, y, orc.MOTION), 2 * g + 18 * 37)
    # first frame of a clip: no predecessor, no difference term
    assert np.array_equal(orc.energy(y, None, orc.MOTION), 2 * g)


def test_motion_weights_are_point6_point4(orc):
    # e = 2 G + 18 D is 5 * (0.4 G + 0.6 * (6 D)): a positive multiple of the
    # paper's 0.4 / 0.6 blend with D brought to the gradient's 0..1530 range.
    rng = np.random.default_rng(9)
    y = rng.integers(0, 256, size=(9, 11)).astype(np.uint8)
    yp = rng.integers(0, 256, size=(9, 11)).astype(np.uint8)
    G = orc.energy(y).astype(np.float64)
    D = np.abs(y.astype(np.float64) - yp)
    blend = 0.4 * G + 0.6 * (D * 1530.0 / 255.0)
    assert np.allclose(orc.energy(y, yp, orc.MOTION), 5.0 * blend)


def test_energy_max_by_vertex_enumeration(orc):
    # |Gx| + |Gy| is convex in the nine pixels, so its maximum over
    # [0, 255]^9 sits on a vertex: enumerate all 512 binary 3x3 patterns.
    best = 0
    for bits in itertools.product((0, 255), repeat=9):
        y = np.array(bits, dtype=np.uint8).reshape(3, 3)
        best = max(best, int(orc.energy(y)[1, 1]))
    assert best == 1530 == orc.energy_max(orc.GRADIENT)
    assert orc.energy_max(orc.MOTION) == 2 * 1530 + 18 * 255 == 7650
