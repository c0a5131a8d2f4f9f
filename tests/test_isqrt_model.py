"""Model of the single-precision path of the kernels' integer square root
(floor(sqrt(q)) for q < 2^40, used by the ASDE test of Sec. 3.2): q as a
float from two conversions and one fused multiply-add, the hardware square
root (within 1 ulp, modelled by the correctly rounded root moved by -1, 0
and +1 ulp), truncation, then one integer comparison each way.  The claim
checked is that the estimate is never off by more than one, so the repaired
value equals floor(sqrt(q)) exactly."""
import math

import numpy as np
import pytest


def model(q: np.ndarray, ulp: int) -> np.ndarray:
    hi = (q >> np.uint64(32)).astype(np.uint32).astype(np.float32)
    lo = (q & np.uint64(0xFFFFFFFF)).astype(np.uint32).astype(np.float32)
    # fma in single precision: the exact sum (representable in double) rounded once
    qf = (hi.astype(np.float64) * 4294967296.0 + lo.astype(np.float64)).astype(np.float32)
    y = np.sqrt(qf)
    if ulp > 0:
        y = np.nextafter(y, np.float32(np.inf))
    elif ulp < 0:
        y = np.nextafter(y, np.float32(0))
    r = y.astype(np.uint64)
    r2 = r * r
    r = np.where(r2 > q, r - np.uint64(1), np.where(r2 + np.uint64(2) * r + np.uint64(1) <= q, r + np.uint64(1), r))
    return r


def exact(q: np.ndarray) -> np.ndarray:
    return np.array([math.isqrt(int(v)) for v in q], dtype=np.uint64)


def cases() -> np.ndarray:
    rng = np.random.default_rng(40)
    lim = 1 << 40
    roots = rng.integers(0, 1 << 20, size=20000, dtype=np.int64)
    near = (roots[:, None] ** 2 + np.arange(-2, 3)[None, :]).ravel()
    near = near[(near >= 0) & (near < lim)]
    rand = rng.integers(0, lim, size=20000, dtype=np.int64)
    small = np.arange(0, 20000, dtype=np.int64)
    top = np.arange(lim - 5000, lim, dtype=np.int64)
    spread = (rng.integers(0, lim, size=20000, dtype=np.int64) >> rng.integers(0, 40, size=20000))
    return np.concatenate([near, rand, small, top, spread]).astype(np.uint64)


@pytest.mark.parametrize("ulp", [-1, 0, 1])
def test_single_precision_path_is_exact(ulp):
    q = cases()
    assert np.array_equal(model(q, ulp), exact(q))
