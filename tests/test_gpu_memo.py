"""GPU parity of seam memorisation (memo_period >= 2: only buffers b with
b mod m == 0 are carved, the others reuse that buffer's removal) against the
oracle's memorisation mode: output pixels, masks, buffer ids and the
per-iteration record are identical, on the plain path, the batched path
(clips with different periods in one call, one and three job groups), the
2-D path and the request server."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def masks_u16(t):
    return t.cpu().numpy().view(np.uint16)


def oracle_kw(kw):
    return dict(mode=kw.get("energy_mode", 1), use_buffer=kw.get("use_buffer", 1), anum=kw.get("alpha_num", 1),
                aden=kw.get("alpha_den", 5), max_buffer=kw.get("max_buffer", 0),
                memo_period=kw.get("memo_period", 0))


@pytest.mark.parametrize("seed,N,H,W,C,Wt,k,kw", [
    (1, 16, 30, 80, 3, 60, 4, dict(memo_period=2, max_buffer=2)),
    (2, 21, 41, 97, 1, 64, 8, dict(memo_period=3, max_buffer=3)),
    (3, 12, 24, 300, 1, 200, 1000, dict(memo_period=2, max_buffer=2)),
    (4, 18, 65, 70, 3, 51, 1, dict(memo_period=4, max_buffer=2, energy_mode=0)),
    (5, 20, 48, 120, 1, 90, 6, dict(memo_period=2)),   # ASDE buffers, scene cut
    (6, 9, 33, 70, 3, 50, 5, dict(memo_period=16, max_buffer=1)),
])
def test_plain_path(ctx, orc, seed, N, H, W, C, Wt, k, kw):
    clip = synth.make_clip(1100 + seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
    res = ctx.retarget(dev(clip), Wt, k, **kw)
    want = orc.retarget(clip, Wt, k, **oracle_kw(kw))
    assert np.array_equal(res["buffer_id"].cpu().numpy(), want["buffer_id"])
    assert np.array_equal(masks_u16(res["masks"]), want["masks"])
    assert np.array_equal(res["out"].cpu().numpy(), want["out"])
    assert np.array_equal(ctx.last_log(), want["log"])


@pytest.mark.parametrize("nstreams", [1, 3])
def test_batched_path(ctx, orc, nstreams):
    specs = [
        (1200, 14, 40, 90, 3, 70, 4, dict(memo_period=2, max_buffer=2)),
        (1201, 10, 65, 33, 1, 24, 16, dict(memo_period=3, max_buffer=1)),
        (1202, 15, 20, 200, 1, 150, 2, dict(max_buffer=3)),                 # no memorisation
        (1203, 12, 36, 64, 3, 40, 1000, dict(memo_period=5, max_buffer=2)),
    ]
    clips, host = [], []
    for seed, N, H, W, C, Wt, k, kw in specs:
        f = synth.make_clip(seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
        host.append((f, Wt, k, kw))
        clips.append(dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=True, **kw))
    ctx.batch_streams(nstreams)
    try:
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
    finally:
        ctx.batch_streams(3)
    for c, (f, Wt, k, kw) in zip(clips, host):
        want = orc.retarget(f, Wt, k, **oracle_kw(kw))
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])
        assert np.array_equal(masks_u16(c["masks"]), want["masks"])
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])


@pytest.mark.parametrize("Wt,Ht", [(40, 27), (30, 36)])
def test_2d_path(ctx, orc, Wt, Ht):
    clip = synth.make_clip(1300, 12, 36, 40, C=3, n_obj=3, lattice=8)
    kw = dict(memo_period=2, max_buffer=2)
    res = ctx.retarget(dev(clip), Wt, 4, want_masks=False, target_height=Ht, **kw)
    want = orc.retarget_2d(clip, Wt, Ht, 4, **oracle_kw(kw))
    assert np.array_equal(res["out"].cpu().numpy(), want["out"])
    assert np.array_equal(res["buffer_id"].cpu().numpy(), want["buffer_id"])


def test_server(orc):
    from paper_1903_03180_amd import scpl
    specs = [(1400, 12, 30, 64, 1, 48, 4, 2), (1401, 10, 40, 50, 3, 36, 8, 3)]
    srv = scpl.Server(0, lanes=2, max_batch=2)
    try:
        tickets, host = [], []
        for seed, N, H, W, C, Wt, k, m in specs:
            f = synth.make_clip(seed, N, H, W, C=C, n_obj=3, lattice=8)
            host.append((f, Wt, k, m))
            clip = dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=True, memo_period=m,
                        max_buffer=2)
            torch.cuda.synchronize()
            tickets.append(srv.submit(clip))
        for t, (f, Wt, k, m) in zip(tickets, host):
            r = srv.wait(t)
            want = orc.retarget(f, Wt, k, max_buffer=2, memo_period=m)
            assert np.array_equal(r["out"].cpu().numpy(), want["out"])
            assert np.array_equal(masks_u16(r["masks"]), want["masks"])
            srv.release(t)
    finally:
        srv.close()


def test_invalid_period_is_refused(ctx):
    from paper_1903_03180_amd import scpl
    f = dev(synth.make_clip(1500, 4, 20, 30, C=1, n_obj=2, lattice=8))
    with pytest.raises(scpl.ScplError):
        ctx.retarget(f, 20, 4, memo_period=-1)


def test_batched_2d(ctx, orc):
    """Batched calls with both dimensions shrinking and memorisation in each
    pass, next to a clip without it."""
    specs = [(1600, 10, 36, 44, 3, 34, 28, dict(memo_period=2, max_buffer=2)),
             (1601, 8, 30, 40, 1, 40, 22, dict(memo_period=3, max_buffer=1)),
             (1602, 9, 28, 48, 1, 36, 28, dict(max_buffer=3))]
    clips, host = [], []
    for seed, N, H, W, C, Wt, Ht, kw in specs:
        f = synth.make_clip(seed, N, H, W, C=C, n_obj=2, lattice=8)
        host.append((f, Wt, Ht, kw))
        clips.append(dict(frames=dev(f), target_width=Wt, target_height=Ht, seams_per_iter=4, **kw))
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    for c, (f, Wt, Ht, kw) in zip(clips, host):
        want = orc.retarget_2d(f, Wt, Ht, 4, **oracle_kw(kw))
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])
