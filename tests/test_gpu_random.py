"""Seeded random clips against the oracle: sizes from one pixel up, luma and
RGB, both energies, with and without buffers, varied alpha, seams per
iteration, buffer-length limits and seam memorisation, some with a target
height; each on the plain path, and all of them in one batched call (several
job groups, uneven shapes side by side) and in one persistent launch; and
frames 450 to 2600 columns wide, plain and batched.  Output frames, masks and buffer
ids must equal the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402


def draw(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 21))
    H = int(rng.choice([1, 2, 3])) if rng.random() < 0.2 else int(rng.integers(4, 48))
    W = int(rng.choice([1, 2, 9])) if rng.random() < 0.2 else int(rng.integers(10, 140))
    C = int(rng.choice([1, 3]))
    Wt = int(rng.integers(max(1, W // 2), W)) if W >= 2 and rng.random() < 0.9 else W
    k = int(rng.choice([1, 2, 4, 16, 1000]))
    kw = dict(energy_mode=int(rng.integers(0, 2)), use_buffer=int(rng.random() < 0.85),
              alpha_num=int(rng.choice([1, 3])), alpha_den=int(rng.choice([5, 20, 50])),
              max_buffer=int(rng.choice([0, 0, 2, 5])), memo_period=int(rng.choice([0, 0, 0, 2])))
    Ht = int(rng.integers(max(1, H // 2), H)) if H >= 4 and rng.random() < 0.25 else 0
    cut = int(rng.integers(1, N)) if N > 2 else None
    f = synth.make_clip(seed, N, H, W, C=C, n_obj=2, cut_at=cut, lattice=4)
    return f, Wt, Ht, k, kw


SEEDS = list(range(7000, 7160))


def oracle_result(orc, f, Wt, Ht, k, kw):
    okw = dict(mode=kw["energy_mode"], use_buffer=kw["use_buffer"], anum=kw["alpha_num"], aden=kw["alpha_den"],
               max_buffer=kw["max_buffer"], memo_period=kw["memo_period"])
    if Ht:
        return orc.retarget_2d(f, Wt, Ht, k, **okw)
    return orc.retarget(f, Wt, k, **okw)


@pytest.fixture(scope="module")
def cases(orc):
    out = []
    for s in SEEDS:
        f, Wt, Ht, k, kw = draw(s)
        out.append((s, f, Wt, Ht, k, kw, oracle_result(orc, f, Wt, Ht, k, kw)))
    return out


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(seed, out, masks, bid, want):
    assert np.array_equal(out.cpu().numpy(), want["out"]), seed
    if masks is not None and want.get("masks") is not None:
        assert np.array_equal(masks.cpu().numpy().view(np.uint16), want["masks"]), seed
    assert np.array_equal(bid.cpu().numpy(), want["buffer_id"]), seed


def test_random_clips_plain(ctx, cases):
    for seed, f, Wt, Ht, k, kw, want in cases:
        extra = dict(kw, target_height=Ht) if Ht else kw
        got = ctx.retarget(dev(f), Wt, k, **extra)
        torch.cuda.synchronize()
        check(seed, got["out"], got["masks"], got["buffer_id"], want)


def test_random_clips_in_one_batch(ctx, cases):
    clips = []
    for seed, f, Wt, Ht, k, kw, want in cases:
        c = dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=not (Ht and Wt < f.shape[2]), **kw)
        if Ht:
            c["target_height"] = Ht
        clips.append(c)
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    for c, (seed, f, Wt, Ht, k, kw, want) in zip(clips, cases):
        check(seed, c["out"], c.get("masks"), c["buffer_id"], want)


def test_random_clips_persistent(cases):
    """The same clips as one persistent launch (its own context), on a
    stream of its own."""
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    try:
        c.batch_mode(scpl.SCPL_BATCH_PERSISTENT)
        clips = []
        for seed, f, Wt, Ht, k, kw, want in cases:
            d = dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=not (Ht and Wt < f.shape[2]), **kw)
            if Ht:
                d["target_height"] = Ht
            clips.append(d)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            c.retarget_batch(clips, stream=s)
        s.synchronize()
        for d, (seed, f, Wt, Ht, k, kw, want) in zip(clips, cases):
            check(seed, d["out"], d.get("masks"), d["buffer_id"], want)
    finally:
        c.close()


def draw_wide(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 8))
    H = int(rng.integers(16, 160))
    W = int(rng.integers(450, 2600))
    C = int(rng.choice([1, 3]))
    Wt = int(rng.integers(int(W * 0.8), W))
    k = int(rng.choice([4, 16, 64]))
    kw = dict(energy_mode=int(rng.integers(0, 2)), alpha_num=1, alpha_den=int(rng.choice([5, 20])),
              max_buffer=int(rng.choice([0, 3])))
    f = synth.make_clip(seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=16)
    return f, Wt, k, kw


WIDE_SEEDS = list(range(7500, 7540))


@pytest.fixture(scope="module")
def wide_cases(orc):
    out = []
    for s in WIDE_SEEDS:
        f, Wt, k, kw = draw_wide(s)
        want = orc.retarget(f, Wt, k, mode=kw["energy_mode"], anum=kw["alpha_num"], aden=kw["alpha_den"],
                            max_buffer=kw["max_buffer"])
        out.append((s, f, Wt, k, kw, want))
    return out


def test_random_wide_clips(ctx, wide_cases):
    """Frames 450 to 2600 columns wide (the column-split DP, several bands
    and compaction passes): plain, then all in one batch."""
    for seed, f, Wt, k, kw, want in wide_cases:
        got = ctx.retarget(dev(f), Wt, k, **kw)
        torch.cuda.synchronize()
        check(seed, got["out"], got["masks"], got["buffer_id"], want)
    clips = [dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=True, **kw)
             for seed, f, Wt, k, kw, want in wide_cases]
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    for c, (seed, f, Wt, k, kw, want) in zip(clips, wide_cases):
        check(seed, c["out"], c["masks"], c["buffer_id"], want)
