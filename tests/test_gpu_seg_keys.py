"""The first DP key rows of a buffer taken from the segmentation's moments:
S1 of the buffer's frames (Sec. 3.2, the sum behind the uniform energy),
less the energies of the frames the window scan read past the buffer's end,
instead of a second pass over the buffer's frames.  The whole retarget must
equal the oracle's for every way the segmentation finishes a buffer:

  * a rejection, with candidate frames scanned past it;
  * the buffer-length limit (max_buffer), with none;
  * the clip's end;
  * a one-frame last buffer that no window scanned (its rows are computed);
  * more carved buffers than a clip keeps rows for (four; the later ones
    computed), and memorised buffers, which keep none;
  * both energies, frames narrower than a tile, two-frame clips;

on the plain path and with all clips in one batched call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402

# (seed, N, H, W, C, Wt, k, cut_at, extra parameters, least number of buffers)
CASES = [
    (900, 40, 36, 70, 1, 50, 4, 20, dict(max_buffer=4), 10),
    (901, 24, 30, 64, 3, 48, 6, 23, {}, 2),                      # one-frame last buffer
    (902, 30, 28, 90, 1, 60, 5, 15, dict(energy_mode=0), 2),
    (903, 20, 25, 6, 1, 4, 1, 10, {}, 2),                        # narrower than a tile
    (904, 36, 22, 50, 1, 35, 3, 18, dict(memo_period=3, max_buffer=3), 12),
    (905, 48, 20, 40, 1, 30, 2, 24, dict(alpha_num=1, alpha_den=10), 7),    # six buffers end in rejections
    (908, 48, 20, 40, 1, 30, 2, 24, dict(alpha_num=1, alpha_den=200), 40),  # one-frame buffers
    (906, 2, 16, 24, 1, 20, 2, None, {}, 1),                     # two frames
    (907, 70, 33, 130, 3, 100, 8, 35, dict(max_buffer=9), 8),
]


def oracle_kw(kw):
    return dict(mode=kw.get("energy_mode", 1), use_buffer=kw.get("use_buffer", 1), anum=kw.get("alpha_num", 1),
                aden=kw.get("alpha_den", 5), max_buffer=kw.get("max_buffer", 0),
                memo_period=kw.get("memo_period", 0))


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cases(orc):
    out = []
    for seed, N, H, W, C, Wt, k, cut, kw, nbuf in CASES:
        f = synth.make_clip(seed, N, H, W, C=C, n_obj=3, cut_at=cut, lattice=8)
        want = orc.retarget(f, Wt, k, **oracle_kw(kw))
        assert int(want["buffer_id"].max()) + 1 >= nbuf, seed
        out.append((f, Wt, k, kw, want))
    return out


def same(got_out, got_masks, got_bid, want):
    assert np.array_equal(got_bid.cpu().numpy(), want["buffer_id"])
    assert np.array_equal(got_masks.cpu().numpy().view(np.uint16), want["masks"])
    assert np.array_equal(got_out.cpu().numpy(), want["out"])


@pytest.mark.parametrize("i", range(len(CASES)))
def test_plain_equals_oracle(ctx, cases, i):
    f, Wt, k, kw, want = cases[i]
    got = ctx.retarget(torch.from_numpy(np.ascontiguousarray(f)).cuda(), Wt, k, **kw)
    torch.cuda.synchronize()
    same(got["out"], got["masks"], got["buffer_id"], want)
    assert np.array_equal(ctx.last_log(), want["log"])


def test_batch_equals_oracle(ctx, cases):
    clips = [dict(frames=torch.from_numpy(np.ascontiguousarray(f)).cuda(), target_width=Wt, seams_per_iter=k,
                  want_masks=True, **kw) for f, Wt, k, kw, _ in cases]
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    log, at = ctx.last_log(), 0
    for c, (_, _, _, _, want) in zip(clips, cases):
        same(c["out"], c["masks"], c["buffer_id"], want)
        n = len(want["log"])
        assert np.array_equal(log[at:at + n], want["log"])
        at += n
    assert at == len(log)
