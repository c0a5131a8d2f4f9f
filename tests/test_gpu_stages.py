"""GPU parity of every stage entry point of libscpl.so against the CPU oracle,
element by element and bit-exact (all arithmetic is integer)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("npx", [1, 15, 16, 17, 4096, 100003])
@pytest.mark.parametrize("offset", [0, 1])
def test_luma(ctx, orc, npx, offset):
    rng = np.random.default_rng(npx + offset)
    rgb = rng.integers(0, 256, size=(npx + offset, 3)).astype(np.uint8)
    want = orc.luma(rgb[offset:])
    d = dev(rgb)[offset:]
    got = host(ctx.luma(d))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 2), (5, 70), (37, 129), (130, 300), (64, 48)])
@pytest.mark.parametrize("mode", [0, 1])
def test_energy(ctx, orc, shape, mode):
    rng = np.random.default_rng(sum(shape) * 3 + mode)
    y = rng.integers(0, 256, size=shape).astype(np.uint8)
    yp = rng.integers(0, 256, size=shape).astype(np.uint8)
    got = host(ctx.energy(dev(y), dev(yp) if mode else None, mode))
    assert np.array_equal(got, orc.energy(y, yp if mode else None, mode))
    if mode:
        got = host(ctx.energy(dev(y), None, mode))
        assert np.array_equal(got, orc.energy(y, None, mode))


# widths span every DP geometry: banded with 2, 4, 8 and 16 columns per
# lane (several wavefronts, bands of 8 to 64 rows, ragged last band) and the
# row-synchronous kernel beyond 8960 columns
DP_SHAPES = [(1, 1), (1, 7), (7, 1), (3, 2), (37, 1100), (70, 2500), (130, 65), (5, 5000), (200, 1920),
             (65, 129), (64, 64), (129, 3), (33, 513), (17, 2240), (45, 4480), (70, 8960), (4, 9500), (3, 20000)]


# hi: tie-heavy energies, the motion energy's maximum, and the largest U the
# 16-bit key rows hold (columns past the width must still never win)
@pytest.mark.parametrize("shape", DP_SHAPES)
@pytest.mark.parametrize("hi", [3, 7650, 16382])
def test_dp(ctx, orc, shape, hi):
    rng = np.random.default_rng(shape[0] * 7 + shape[1] + hi)
    u = rng.integers(0, hi + 1, size=shape).astype(np.int32)
    ce, lab, d = ctx.dp(dev(u))
    oce, olab, od = orc.dp(u)
    assert np.array_equal(host(ce), oce[-1])
    assert np.array_equal(host(lab), olab[-1])
    assert np.array_equal(host(d), od)


@pytest.mark.parametrize("bad", [-1, 16383, 1 << 30])
def test_dp_refuses_energy_outside_key_range(ctx, bad):
    """U outside [0, 16382] does not fit the 16-bit key rows: the call
    returns SCPL_ERR_INVALID_ARG and leaves the outputs untouched."""
    from paper_1903_03180_amd import scpl
    u = np.full((9, 40), 5, dtype=np.int32)
    u[4, 17] = bad
    ce = torch.full((40,), -7, dtype=torch.int32, device="cuda")
    lab = torch.full((40,), -7, dtype=torch.int32, device="cuda")
    d = torch.full((9, 40), 9, dtype=torch.int8, device="cuda")
    du = dev(u)
    st = scpl.scpl_dp(ctx.h, 9, 40, du.data_ptr(), ce.data_ptr(), lab.data_ptr(), d.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
    assert st == scpl.SCPL_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((ce == -7).all()) and bool((lab == -7).all()) and bool((d == 9).all())
    # the context stays usable
    u[4, 17] = 16382
    ce2, _, _ = ctx.dp(dev(u))
    assert ce2.shape == (40,)


# widths above 10176 hold the selection keys (16 bytes per column) in global
# memory instead of the 159 KiB of LDS
@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (5, 6), (60, 1920), (9, 3000), (40, 4100), (3, 12000),
                                   (2, 20000)])
@pytest.mark.parametrize("k", [1, 3, 16, 10**6])
def test_select(ctx, orc, shape, k):
    rng = np.random.default_rng(shape[1] + k % 1000)
    u = rng.integers(0, 4, size=shape).astype(np.int32)
    oce, olab, od = orc.dp(u)
    W = shape[1]
    for limit in sorted({W, max(1, W // 3), 1}):
        ch, peff = ctx.select(dev(oce[-1]), dev(olab[-1]), k, limit)
        och, opeff = orc.select(oce[-1], olab[-1], k, limit)
        assert peff == opeff
        assert np.array_equal(host(ch), och)


@pytest.mark.parametrize("shape", [(1, 5), (2, 9), (64, 64), (65, 70), (200, 300), (129, 1920), (1080, 256)])
@pytest.mark.parametrize("k", [1, 5, 32])
def test_backtrack(ctx, orc, shape, k):
    rng = np.random.default_rng(shape[0] + 13 * shape[1] + k)
    u = rng.integers(0, 20, size=shape).astype(np.int32)
    oce, olab, od = orc.dp(u)
    och, _ = orc.select(oce[-1], olab[-1], k)
    seams = ctx.backtrack(dev(od), dev(och))
    assert np.array_equal(host(seams), orc.backtrack(od, och))


def _clip(seed, N, H, W, C=1, cut=None):
    from paper_1903_03180_amd import synth
    return synth.make_clip(seed, N, H, W, C=C, n_obj=3, cut_at=cut, lattice=8, max_speed=5)


@pytest.mark.parametrize("alpha", [(3, 20), (1, 5), (1, 4), (1, 40), (0, 1)])
@pytest.mark.parametrize("mode", [1, 0])
def test_segment(ctx, orc, alpha, mode):
    Y = _clip(71, 150, 21, 35, cut=90)
    bid, tr = ctx.segment(dev(Y), energy_mode=mode, alpha_num=alpha[0], alpha_den=alpha[1])
    obid, otr = orc.segment(Y, mode, 1, alpha[0], alpha[1])
    assert np.array_equal(bid, obid)
    assert np.array_equal(tr, otr)


def test_segment_max_buffer_and_off(ctx, orc):
    Y = _clip(72, 40, 16, 20)
    for mb in (1, 2, 7, 64, 65):
        bid, tr = ctx.segment(dev(Y), alpha_num=1, alpha_den=1, max_buffer=mb)
        obid, otr = orc.segment(Y, 1, 1, 1, 1, mb)
        assert np.array_equal(bid, obid) and np.array_equal(tr, otr)
    bid, _ = ctx.segment(dev(Y), use_buffer=0)
    assert bid.tolist() == list(range(40))


from paper_1903_03180_amd.scpl import DP_CHUNKED  # noqa: E402
from paper_1903_03180_amd.scpl import DP_GEOMETRIES as GEOMETRIES  # noqa: E402


def test_dp_extreme_values_at_the_border(ctx, orc):
    """U at its maximum next to the right border and zero elsewhere: the
    0xffff columns past the width sit beside the costliest real column."""
    for shape in [(50, 1920), (200, 77), (9, 6001)]:
        u = np.zeros(shape, dtype=np.int32)
        u[:, -1] = 16382
        u[::3, -2] = 16382
        ce, lab, d = ctx.dp(dev(u))
        oce, olab, od = orc.dp(u)
        assert np.array_equal(host(ce), oce[-1]) and np.array_equal(host(d), od), shape


@pytest.mark.parametrize("geom", [g + (ex,) for g in GEOMETRIES for ex in (0, 1)])
def test_dp_every_geometry(ctx, orc, geom):
    """Every DP geometry (columns per lane, halo / band rows, prefetch) gives the
    oracle's result; widths a geometry cannot hold fall back to the default
    and must agree too."""
    ctx.dp_geometry(*geom)
    try:
        for shape in [(3, 1), (40, 333), (130, 1000), (77, 1920), (20, 3100), (9, 6000)]:
            rng = np.random.default_rng(shape[1] + geom[0])
            u = rng.integers(0, 40, size=shape).astype(np.int32)
            ce, lab, d = ctx.dp(dev(u))
            oce, olab, od = orc.dp(u)
            assert np.array_equal(host(ce), oce[-1]), shape
            assert np.array_equal(host(lab), olab[-1]), shape
            assert np.array_equal(host(d), od), shape
    finally:
        ctx.dp_geometry(0)


CHUNKED = DP_CHUNKED + [(4, 16, 8, 16, 64), (2, 8, 16, 8, 16), (4, 8, 8, 32, 96), (4, 16, 16, 20, 64),
                        (4, 16, 16, 48, 96)]


@pytest.mark.parametrize("geom", [g + (ex,) for g in CHUNKED for ex in (0, 1)])
def test_dp_chunked(ctx, orc, geom):
    """Column-split DP (one launch per R rows, a workgroup per P columns):
    the oracle's result for heights below, at and above multiples of R and
    widths below, at and above multiples of P, with the extreme key 16382
    at the borders."""
    q, hb, pf, R, P, ex = geom
    ctx.dp_geometry(q, hb, pf, ex)
    ctx.dp_chunking(R, P)
    try:
        g = ctx.dp_chosen(4096)
        assert (g["chunk_rows"], g["chunk_cols"]) == (R, P)
        for shape in [(1, 7), (2, 1), (R, P), (R + 1, P - q), (2 * R - 1, 2 * P + 5), (3 * R, 3 * P),
                      (130, 1000), (77, 1920), (20, 3100)]:
            rng = np.random.default_rng(shape[0] * 7 + shape[1] + q)
            u = rng.integers(0, 40, size=shape).astype(np.int32)
            u[:, 0] = 16382
            u[::2, -1] = 16382
            ce, lab, d = ctx.dp(dev(u))
            oce, olab, od = orc.dp(u)
            assert np.array_equal(host(ce), oce[-1]), shape
            assert np.array_equal(host(lab), olab[-1]), shape
            assert np.array_equal(host(d), od), shape
    finally:
        ctx.dp_geometry(0)


def test_autotune_then_parity(ctx, orc):
    q, hb, pf, ex, us = ctx.autotune_dp(256, 1920, n_jobs=3)
    assert (q, hb, pf) in GEOMETRIES and ex in (0, 1) and us > 0
    rng = np.random.default_rng(3)
    u = rng.integers(0, 7651, size=(90, 1920)).astype(np.int32)
    ce, lab, d = ctx.dp(dev(u))
    oce, olab, od = orc.dp(u)
    assert np.array_equal(host(ce), oce[-1]) and np.array_equal(host(d), od)


@pytest.mark.parametrize("n,H,W,mode,prev", [(1, 9, 13, 1, False), (2, 17, 30, 1, True), (5, 33, 65, 0, False),
                                             (64, 20, 24, 1, False), (65, 20, 24, 1, True), (70, 16, 40, 0, True),
                                             (12, 1, 1, 1, True)])
@pytest.mark.parametrize("alpha", [(1, 5), (3, 20), (1, 50)])
def test_asde(ctx, orc, n, H, W, mode, prev, alpha):
    Y = _clip(81 + n, n + 1, H, W, cut=n // 2 + 1)
    first = 1
    frames, before = Y[first:], Y[0]
    s1 = np.zeros((H, W), dtype=np.uint64)
    s2 = np.zeros((H, W), dtype=np.uint64)
    for t in range(n):
        p = (frames[t - 1] if t else before) if mode == 1 and (t or prev) else None
        e = orc.energy(frames[t], p, mode).astype(np.uint64)
        s1 += e
        s2 += e * e
    S = orc.asde_sum(s1, s2, n)
    rej = orc.reject(S, n, H * W, orc.energy_max(mode), alpha[0], alpha[1])
    gS, grej = ctx.asde(dev(frames), dev(before) if prev else None, energy_mode=mode, alpha_num=alpha[0],
                        alpha_den=alpha[1])
    assert gS == S and grej == rej


@pytest.mark.parametrize("n,prev", [(700, False), (900, True)])
def test_asde_large_moments(ctx, orc, n, prev):
    """A random frame shown twice, then black, over and over: the per-pixel
    n^2-scaled variances n S2 - S1^2 spread across 2^40, so both the
    single-precision and the double-precision paths of the kernel's integer
    square root are taken, against the oracle's exact sums."""
    H, W = 12, 20
    rng = np.random.default_rng(n)
    X = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    Y = np.stack([X if t % 3 else np.zeros_like(X) for t in range(n + 1)])
    frames, before = Y[1:], Y[0]
    s1 = np.zeros((H, W), dtype=np.uint64)
    s2 = np.zeros((H, W), dtype=np.uint64)
    for t in range(n):
        p = (frames[t - 1] if t else before) if (t or prev) else None
        e = orc.energy(frames[t], p, 1).astype(np.uint64)
        s1 += e
        s2 += e * e
    q = n * s2.astype(object) - s1.astype(object) ** 2
    assert min(q.flat) < 2 ** 40 < max(q.flat)
    S = orc.asde_sum(s1, s2, n)
    rej = orc.reject(S, n, H * W, orc.energy_max(1), 1, 5)
    gS, grej = ctx.asde(dev(frames), dev(before) if prev else None, energy_mode=1, alpha_num=1, alpha_den=5)
    assert gS == S and grej == rej


@pytest.mark.parametrize("shape,kk,C", [((1, 5), 2, 1), ((40, 70), 7, 3), ((130, 300), 60, 1), ((9, 2000), 1500, 3),
                                        ((64, 64), 0, 1)])
def test_compact(ctx, orc, shape, kk, C):
    H, W = shape
    rng = np.random.default_rng(H + W + kk)
    u = rng.integers(0, 9, size=shape).astype(np.int32)
    oce, olab, od = orc.dp(u)
    och, _ = orc.select(oce[-1], olab[-1], max(kk, 1), max(kk, 1))
    seams = orc.backtrack(od, och)[:kk] if kk else np.zeros((0, H), dtype=np.int32)
    kk = seams.shape[0]
    frame = rng.integers(0, 256, size=(H, W, C) if C == 3 else (H, W)).astype(np.uint8)
    want = np.stack([np.delete(frame[i], seams[:, i], axis=0) for i in range(H)])
    got = ctx.compact(dev(frame), dev(seams.astype(np.int32)))
    assert np.array_equal(host(got), want)
