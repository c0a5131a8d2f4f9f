"""GPU parity of the whole retarget (plain path and batched path) against the
CPU oracle: output pixels, masks, buffer ids and the per-iteration record
(W_r, P_eff, k_iter) must be identical.  At the full 1080p and 4K sizes the
oracle cannot run the whole clip in seconds, so there the segmentation and
the first iteration of every buffer are compared exactly and the rest is
checked through properties that hold at any size."""
import os

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


def compare(ctx, orc, frames, Wt, k, **kw):
    res = ctx.retarget(dev(frames), Wt, k, **kw)
    okw = dict(mode=kw.get("energy_mode", 1), use_buffer=kw.get("use_buffer", 1), anum=kw.get("alpha_num", 1),
               aden=kw.get("alpha_den", 5), max_buffer=kw.get("max_buffer", 0))
    want = orc.retarget(frames, Wt, k, **okw)
    assert np.array_equal(res["buffer_id"].cpu().numpy(), want["buffer_id"])
    assert np.array_equal(masks_u16(res["masks"]), want["masks"])
    assert np.array_equal(res["out"].cpu().numpy(), want["out"])
    assert np.array_equal(ctx.last_log(), want["log"])
    return res, want


def test_cfg1_single_image(ctx, orc):
    img = synth.image_cfg1(1)
    compare(ctx, orc, img[None], 56, 8, energy_mode=0, use_buffer=0)


@pytest.mark.parametrize("seed,N,H,W,C,Wt,k", [
    (1, 12, 30, 52, 3, 38, 3),
    (2, 20, 41, 97, 1, 60, 8),
    (3, 9, 64, 64, 3, 33, 16),
    (4, 16, 70, 130, 1, 100, 1),
    (5, 10, 17, 300, 3, 200, 1000),
    (6, 7, 129, 75, 1, 70, 2),
    (7, 14, 96, 160, 3, 120, 4),
])
def test_small_clips_motion(ctx, orc, seed, N, H, W, C, Wt, k):
    clip = synth.make_clip(300 + seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
    compare(ctx, orc, clip, Wt, k)


@pytest.mark.parametrize("alpha", [(3, 20), (1, 5), (1, 4)])
def test_alpha_sweep_with_pan(ctx, orc, alpha):
    clip = synth.make_clip(77, 24, 48, 120, C=1, n_obj=4, pan_div=2, lattice=16)
    compare(ctx, orc, clip, 90, 6, alpha_num=alpha[0], alpha_den=alpha[1])


@pytest.mark.parametrize("kw", [dict(use_buffer=0), dict(energy_mode=0), dict(energy_mode=0, use_buffer=0),
                                dict(max_buffer=3), dict(alpha_num=0)])
def test_modes(ctx, orc, kw):
    clip = synth.make_clip(88, 10, 33, 70, C=3, n_obj=3, cut_at=5, lattice=8)
    compare(ctx, orc, clip, 50, 5, **kw)


@pytest.mark.parametrize("shape,Wt,k", [((1, 1, 1), 1, 1), ((3, 1, 9), 4, 2), ((2, 9, 1), 1, 3), ((4, 5, 6), 6, 2),
                                        ((2, 1, 3000), 1000, 700), ((3, 5, 3000), 1200, 1500),
                                        ((2, 7, 9100), 9000, 40)])
def test_degenerate(ctx, orc, shape, Wt, k):
    rng = np.random.default_rng(sum(shape))
    clip = rng.integers(0, 256, size=shape).astype(np.uint8)
    compare(ctx, orc, clip, Wt, k)


@pytest.mark.parametrize("nstreams", [1, 2, 3, 8])
def test_batch_equals_oracle_and_plain(ctx, orc, nstreams):
    clips = [
        dict(frames=synth.make_clip(500, 12, 40, 90, C=3, n_obj=3, cut_at=6, lattice=8), target_width=70,
             seams_per_iter=4),
        dict(frames=synth.make_clip(501, 9, 65, 33, C=1, n_obj=2, lattice=8), target_width=24, seams_per_iter=16),
        dict(frames=synth.image_cfg1(1)[None], target_width=56, seams_per_iter=8, energy_mode=0, use_buffer=0),
        dict(frames=synth.make_clip(502, 15, 20, 200, C=1, n_obj=3, cut_at=4, lattice=8), target_width=150,
             seams_per_iter=2, alpha_num=3, alpha_den=20),
    ]
    host = [c["frames"] for c in clips]
    for c in clips:
        c["frames"] = dev(c["frames"])
        c["want_masks"] = True
    ctx.batch_streams(nstreams)
    try:
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
    finally:
        ctx.batch_streams(3)
    for c, fr in zip(clips, host):
        kw = dict(mode=c.get("energy_mode", 1), use_buffer=c.get("use_buffer", 1), anum=c.get("alpha_num", 1),
                  aden=c.get("alpha_den", 5))
        want = orc.retarget(fr, c["target_width"], c["seams_per_iter"], **kw)
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(masks_u16(c["masks"]), want["masks"])
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])


@pytest.mark.parametrize("seed,N,H,W,C,Wt,Ht,k", [
    (1, 12, 30, 52, 3, 38, 0, 3),
    (2, 9, 70, 300, 1, 220, 0, 6),
    (3, 7, 35, 60, 3, 45, 28, 3),   # width and height: the height pass's temporaries too
    (4, 8, 40, 30, 1, 30, 29, 4),   # height only
])
def test_caller_workspace_equals_own(ctx, orc, seed, N, H, W, C, Wt, Ht, k):
    """scpl_retarget with a caller's workspace of exactly
    scpl_workspace_size bytes gives the result of the context's own
    workspace (and the oracle's); the region is left to the caller."""
    from paper_1903_03180_amd import scpl
    clip = synth.make_clip(630 + seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
    d = dev(clip)
    kw = dict(target_height=Ht) if Ht else {}
    want_masks = not (Ht and Wt < W)
    p = scpl.params_for(d, Wt, k, **kw)
    nbytes = scpl.workspace_size(p)
    ws = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    a = ctx.retarget(d, Wt, k, want_masks=want_masks, workspace=ws, **kw)
    b = ctx.retarget(d, Wt, k, want_masks=want_masks, **kw)
    torch.cuda.synchronize()
    assert torch.equal(a["out"], b["out"]) and torch.equal(a["buffer_id"], b["buffer_id"])
    if want_masks:
        assert torch.equal(a["masks"], b["masks"])
    want = orc.retarget_2d(clip, Wt, Ht, k) if Ht else orc.retarget(clip, Wt, k)
    assert np.array_equal(a["out"].cpu().numpy(), want["out"])


def test_caller_workspace_too_small_or_misaligned(ctx):
    from paper_1903_03180_amd import scpl
    d = dev(synth.make_clip(640, 5, 20, 40, C=1, n_obj=2, lattice=8))
    nbytes = scpl.workspace_size(scpl.params_for(d, 30, 4))
    ws = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(scpl.ScplError) as e:
        ctx.retarget(d, 30, 4, workspace=ws[:nbytes - 1])
    assert e.value.status == scpl.SCPL_ERR_INVALID_ARG
    with pytest.raises(scpl.ScplError) as e:
        ctx.retarget(d, 30, 4, workspace=ws[16:16 + nbytes])
    assert e.value.status == scpl.SCPL_ERR_INVALID_ARG
    ctx.retarget(d, 30, 4, workspace=ws[256:256 + nbytes])


@pytest.mark.parametrize("seed,N,H,W,C,Wt,k,kw", [
    (1, 48, 36, 100, 1, 70, 4, dict(alpha_num=1, alpha_den=2)),   # one 48-frame buffer: 3 pieces of 16 frames
    (2, 70, 20, 64, 3, 44, 3, dict(alpha_num=1, alpha_den=2, max_buffer=40)),  # 40 + 30 frames, RGB
    (3, 2, 6, 12000, 1, 11900, 40, {}),   # selection keys in global memory (W > 10176)
    (4, 3, 300, 8000, 1, 7950, 32, {}),   # 96-row bands (selection LDS of 159 KiB)
    (5, 3, 450, 3000, 1, 2950, 16, {}),   # 96-row bands under a 63 KiB selection LDS
])
def test_paths_full_sizes_reach(ctx, orc, seed, N, H, W, C, Wt, k, kw):
    """Paths the full-size workloads take that the small clips do not:
    buffers longer than 32 frames (the refresh's sum over several
    16-frame pieces of the pixel-major luma), widths whose selection keys do
    not fit LDS, and band heights above 32 rows.  Against the oracle."""
    clip = synth.make_clip(650 + seed, N, H, W, C=C, n_obj=3, lattice=8)
    res, want = compare(ctx, orc, clip, Wt, k, **kw)
    if seed == 1:
        assert np.bincount(want["buffer_id"]).tolist() == [48]
    if seed == 2:
        assert np.bincount(want["buffer_id"]).tolist() == [40, 30]


def test_repeat_runs_identical(ctx):
    clip = dev(synth.make_clip(9, 16, 72, 128, C=3, n_obj=3, cut_at=8, lattice=8))
    a = ctx.retarget(clip, 90, 8)
    b = ctx.retarget(clip, 90, 8)
    assert torch.equal(a["out"], b["out"]) and torch.equal(a["masks"], b["masks"])


# ------------------------------------------------------------- full sizes

def removed_carved_columns(mask_row, r):
    alive = (mask_row == 0) | (mask_row > r)
    pos = np.cumsum(alive) - 1
    return pos[mask_row == r + 1]


def check_full_size(orc, frames, res, Wt, k, mode, anum, aden, n_first=None):
    """Exact: segmentation, and iteration 0 of each buffer (U from the
    oracle's energy over the buffer's frames, the oracle's DP, select and
    backtrack).  Properties: uniform width, output = input without masked
    pixels, one mask per buffer, k_iter 8-connected seams per iteration."""
    N, H, W = frames.shape[:3]
    Y = orc.luma(frames) if frames.ndim == 4 else frames
    obid, _ = orc.segment(Y, mode, 1, anum, aden)
    bid = res["buffer_id"].cpu().numpy()
    assert np.array_equal(bid, obid)
    masks = masks_u16(res["masks"])
    out = res["out"].cpu().numpy()
    assert np.all((masks > 0).sum(axis=2) == W - Wt)
    for t in range(N):
        keep = masks[t] == 0
        assert np.array_equal(out[t], frames[t][keep].reshape(out[t].shape))
        if t and bid[t] == bid[t - 1]:
            assert np.array_equal(masks[t], masks[t - 1])
    for b in np.unique(bid):
        idx = np.nonzero(bid == b)[0]
        t0, T = int(idx[0]), len(idx)
        if n_first is not None and b >= n_first:
            break
        ghost = 1 if (mode == 1 and t0 > 0) else 0
        acc = np.zeros((H, W), dtype=np.int64)
        for t in range(t0, t0 + T):
            prev = Y[t - 1] if (t > t0 or ghost) else None
            acc += orc.energy(Y[t], prev, mode)
        U = (acc // T).astype(np.int32)
        ce, lab, d = orc.dp(U)
        ch, _ = orc.select(ce[-1], lab[-1], k, W - Wt)
        seams = orc.backtrack(d, ch)
        m = masks[t0]
        got = np.stack([np.nonzero(m[i] == 1)[0] for i in range(H)], axis=1)
        assert np.array_equal(got, seams)
        # later iterations: k_iter 8-connected seams on the carved grid
        r = 1
        while True:
            cols = [removed_carved_columns(m[i], r) for i in range(H)]
            if len(cols[0]) == 0:
                break
            assert all(len(c) == len(cols[0]) for c in cols)
            s = np.stack(cols, axis=1)
            assert np.all(np.abs(np.diff(s, axis=1)) <= 1)
            r += 1


def test_1080p_clip_full_size(ctx, orc):
    frames = synth.clip_1080p(2)
    res = ctx.retarget(dev(frames), 1440, 16)
    torch.cuda.synchronize()
    assert res["n_buffers"] >= 2  # the scene cut at frame 60 breaks the buffer
    bid = res["buffer_id"].cpu().numpy()
    assert bid[60] != bid[59]
    check_full_size(orc, frames, res, 1440, 16, 1, 1, 5)


@pytest.mark.parametrize("alpha", [(3, 20), (1, 5), (1, 4)])
def test_4k_clip_full_size(ctx, orc, alpha):
    frames = synth.clip_4k(3)
    res = ctx.retarget(dev(frames), 2880, 32, alpha_num=alpha[0], alpha_den=alpha[1])
    torch.cuda.synchronize()
    check_full_size(orc, frames, res, 2880, 32, 1, alpha[0], alpha[1], n_first=1)


@pytest.mark.parametrize("which", ["1080p", "4k"])
def test_full_size_with_benchmarked_chunked_dp(ctx, orc, which):
    """The full-size single clips with the column-split DP the autotuner
    picks for them in the benchmark ((4,16,8), 256 rows x 384 columns per
    workgroup): bit-identical to a single-workgroup DP (8,16,8), and
    segmentation plus the first iteration of the first buffer exact against
    the oracle."""
    if which == "1080p":
        frames, Wt, k = synth.clip_1080p(2), 1440, 16
    else:
        frames, Wt, k = synth.clip_4k(3), 2880, 32
    d = dev(frames)
    try:
        ctx.dp_geometry(8, 16, 8, 1)
        ref = ctx.retarget(d, Wt, k)
        ctx.dp_geometry(4, 16, 8, 1)
        ctx.dp_chunking(256, 384)
        res = ctx.retarget(d, Wt, k)
        torch.cuda.synchronize()
    finally:
        ctx.dp_geometry(0)
    assert torch.equal(res["out"], ref["out"])
    assert torch.equal(res["masks"], ref["masks"])
    assert torch.equal(res["buffer_id"], ref["buffer_id"])
    check_full_size(orc, frames, res, Wt, k, 1, 1, 5, n_first=1)


@pytest.mark.parametrize("geom", [(4, 8, 16, 1), (4, 16, 8, 0), (8, 16, 8, 1), (8, 32, 4, 0), (32, 0, 2, 1)])
def test_forced_geometry_retarget(ctx, orc, geom):
    clip = synth.make_clip(610, 8, 40, 300, C=3, n_obj=3, cut_at=4, lattice=8)
    ctx.dp_geometry(*geom)
    try:
        compare(ctx, orc, clip, 220, 6)
    finally:
        ctx.dp_geometry(0)


@pytest.mark.parametrize("geom", [(4, 16, 8, 1, 32, 64), (2, 8, 16, 0, 16, 96), (4, 16, 8, 1, 128, 640),
                                  (4, 16, 16, 1, 40, 96), (4, 16, 16, 0, 64, 128)])
def test_chunked_geometry_retarget(ctx, orc, geom):
    """Whole retargets with a column-split DP (many row chunks and
    workgroups for the small R, P), against the oracle."""
    clip = synth.make_clip(611, 8, 70, 300, C=3, n_obj=3, cut_at=4, lattice=8)
    q, hb, pf, ex, R, P = geom
    ctx.dp_geometry(q, hb, pf, ex)
    ctx.dp_chunking(R, P)
    try:
        compare(ctx, orc, clip, 220, 6)
    finally:
        ctx.dp_geometry(0)


@pytest.mark.parametrize("shape,Wt", [((3, 144, 176), 140), ((2, 144, 176), 105), ((2, 48, 64), 38)])
def test_raw_baseline_matches_oracle(ctx, orc, shape, Wt):
    """The paper's comparison "Raw": classic seam carving of every frame on
    its own (one seam per iteration, gradient energy, no buffer), at Table 1
    shapes and ratios."""
    N, H, W = shape
    clip = synth.make_clip(950 + W, N, H, W, C=3, n_obj=3, lattice=8)
    compare(ctx, orc, clip, Wt, 1, energy_mode=0, use_buffer=0)


def test_uncapped_one_seam_per_parent(ctx, orc):
    """k >= W: every parent's least child leaves in each iteration (eq. 6
    taken literally)."""
    clip = synth.make_clip(960, 12, 40, 96, C=1, n_obj=3, cut_at=6, lattice=8)
    compare(ctx, orc, clip, 60, 96)


# --------------------------------------------------- height and 2-D retargeting

def compare_2d(ctx, orc, frames, Wt, Ht, k, **kw):
    want_masks = not (Wt < frames.shape[2] and Ht < frames.shape[1])
    res = ctx.retarget(dev(frames), Wt, k, want_masks=want_masks, target_height=Ht, **kw)
    okw = dict(mode=kw.get("energy_mode", 1), use_buffer=kw.get("use_buffer", 1), anum=kw.get("alpha_num", 1),
               aden=kw.get("alpha_den", 5), max_buffer=kw.get("max_buffer", 0))
    want = orc.retarget_2d(frames, Wt, Ht, k, **okw)
    assert np.array_equal(res["out"].cpu().numpy(), want["out"])
    assert np.array_equal(res["buffer_id"].cpu().numpy(), want["buffer_id"])
    assert np.array_equal(ctx.last_log(), want["log"])
    if want_masks:
        assert np.array_equal(masks_u16(res["masks"]), want["masks"])


@pytest.mark.parametrize("seed,N,H,W,C,Wt,Ht,k", [
    (1, 8, 40, 30, 3, 30, 29, 4),      # height only
    (2, 12, 64, 48, 1, 48, 40, 16),
    (3, 7, 35, 60, 3, 45, 28, 3),      # both: width first, then height
    (4, 5, 90, 33, 1, 20, 70, 1000),
])
def test_height_and_2d(ctx, orc, seed, N, H, W, C, Wt, Ht, k):
    clip = synth.make_clip(700 + seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
    compare_2d(ctx, orc, clip, Wt, Ht, k)


def test_batch_mixed_directions(ctx, orc):
    specs = [(710, 9, 30, 50, 3, 40, 30), (711, 6, 44, 26, 1, 26, 33), (712, 10, 28, 40, 1, 31, 20)]
    clips, host = [], []
    for seed, N, H, W, C, Wt, Ht in specs:
        f = synth.make_clip(seed, N, H, W, C=C, n_obj=2, cut_at=N // 2, lattice=8)
        host.append((f, Wt, Ht))
        clips.append(dict(frames=dev(f), target_width=Wt, target_height=Ht, seams_per_iter=6))
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    for c, (f, Wt, Ht) in zip(clips, host):
        want = orc.retarget_2d(f, Wt, Ht, 6)
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])


def test_2d_masks_are_refused(ctx):
    from paper_1903_03180_amd import scpl
    f = dev(synth.make_clip(720, 4, 30, 30, C=1, n_obj=2, lattice=8))
    with pytest.raises(scpl.ScplError):
        ctx.retarget_batch([dict(frames=f, target_width=20, target_height=20, seams_per_iter=4, want_masks=True)])


def test_1080p_batch_as_benchmarked(ctx, orc):
    """The benchmark's launch configuration at full size: several 1080p
    clips in one batched call, three stream groups, autotuned DP geometry.
    Every clip equals its plain-path result bit for bit; the first clip is
    also checked against the oracle (segmentation, first iteration of every
    buffer) and through the invariants."""
    seeds = [2000, 2001, 2002]
    frames = [synth.clip_1080p(s) for s in seeds]
    ctx.batch_streams(3)
    ctx.autotune_dp(1080, 1920, n_jobs=3 * len(seeds))
    try:
        clips = [dict(frames=dev(f), target_width=1440, seams_per_iter=16, want_masks=True) for f in frames]
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
        for c in clips:
            solo = ctx.retarget(c["frames"], 1440, 16)
            assert torch.equal(c["out"], solo["out"]) and torch.equal(c["masks"], solo["masks"])
            assert torch.equal(c["buffer_id"], solo["buffer_id"])
        res = dict(out=clips[0]["out"], masks=clips[0]["masks"], buffer_id=clips[0]["buffer_id"])
        check_full_size(orc, frames[0], res, 1440, 16, 1, 1, 5)
    finally:
        ctx.dp_geometry(0)


def test_uneven_mix_batch_equals_plain(ctx):
    """Clips of the uneven mix (luma, widths up to 2560, 30-240 frames) in
    one batch give exactly their plain-path results."""
    specs = [s for s in synth.batch_mix_specs(64)][:6]
    clips = [dict(frames=dev(synth.clip_from_spec(s)), target_width=s.Wt, seams_per_iter=16) for s in specs]
    ctx.retarget_batch(clips)
    torch.cuda.synchronize()
    for c, s in zip(clips, specs):
        solo = ctx.retarget(c["frames"], s.Wt, 16, want_masks=False)
        assert torch.equal(c["out"], solo["out"]), s
        assert torch.equal(c["buffer_id"], solo["buffer_id"]), s


def test_profile_kinds_bracket_only_the_chosen_kernels(ctx):
    from paper_1903_03180_amd import scpl
    clip = dev(synth.make_clip(620, 8, 30, 80, C=3, n_obj=2, lattice=8))
    try:
        ctx.profile(True, kinds=["dp"])
        ctx.retarget_batch([dict(frames=clip, target_width=60, seams_per_iter=4)])
        prof = ctx.profile_read()
        assert prof["dp"][1] > 0 and prof["dp"][0] > 0
        assert all(n == 0 for k, (ms, n) in prof.items() if k != "dp")
        ctx.profile(True)
        ctx.retarget_batch([dict(frames=clip, target_width=60, seams_per_iter=4)])
        prof = ctx.profile_read()
        assert all(prof[k][1] > 0 for k in ("luma", "segment", "dp", "select", "update", "gather"))
    finally:
        ctx.profile(False)
    with pytest.raises(scpl.ScplError):
        scpl._check(scpl.scpl_profile_kinds(ctx.h, 1 << len(scpl.KERNELS)), "scpl_profile_kinds")


@pytest.mark.parametrize("upd,ref,borg,gat,fuse", [
    (0, 0, 0, 0, 0), (1, 0, 0, 0, 0), (2, 0, 0, 0, 0), (3, 0, 0, 0, 0), (4, 0, 0, 0, 0), (5, 0, 0, 0, 0),
    (6, 0, 0, 0, 0), (0, 1, 0, 0, 0), (0, 2, 0, 0, 0), (0, 0, 1, 0, 0), (0, 0, 2, 0, 0), (0, 0, 0, 1, 0),
    (0, 0, 0, 2, 0), (0, 0, 0, 3, 0), (0, 0, 0, 4, 0), (4, 2, 2, 3, 0), (5, 1, 1, 2, 0), (0, 0, 0, 0, 1),
    (0, 0, 0, 0, 2), (3, 1, 2, 2, 1), (3, 0, 0, 4, 1)])
def test_kernel_variants_retarget(ctx, orc, upd, ref, borg, gat, fuse):
    """Every compaction variant (rows per workgroup x columns per pass, so
    widths of several passes), refresh variant, band-origin variant and
    gather variant (frames per pass; buffers whose length is not a multiple
    of it), and the fill and compaction fused per band, on the plain path
    and in a batch, against the oracle."""
    clip = synth.make_clip(660, 6, 50, 2600, C=1, n_obj=3, cut_at=3, lattice=16)
    small = synth.make_clip(661, 9, 40, 300, C=3, n_obj=3, cut_at=4, lattice=8)
    ctx.kernel_variants(upd, ref, borg, gat, fuse)
    try:
        compare(ctx, orc, clip, 2450, 20)
        clips = [dict(frames=dev(clip), target_width=2450, seams_per_iter=20, want_masks=True),
                 dict(frames=dev(small), target_width=210, seams_per_iter=6, want_masks=True)]
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
    finally:
        ctx.kernel_variants()
    for c, f, wt, k in zip(clips, (clip, small), (2450, 210), (20, 6)):
        want = orc.retarget(f, wt, k)
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(masks_u16(c["masks"]), want["masks"])


# (seed, N, H, W, C, Wt, k)
STREAMED = [
    (670, 7, 24, 320, 3, 240, 8),       # 960-byte rows, 720-byte output rows: streamed
    (671, 5, 20, 2048, 1, 1600, 64),    # streamed
    (672, 5, 12, 3840, 3, 2880, 96),    # 11,520-byte rows: the loaders' wider register set
    (673, 3, 10, 6000, 3, 5400, 100),   # 18,000-byte rows: gathered as by variant 0
    (674, 9, 30, 300, 3, 210, 6),       # 900-byte rows (not 16-byte multiples): as variant 0
]


@pytest.mark.parametrize("want_masks", [True, False])
def test_gather_streamed_rows(ctx, orc, want_masks):
    """Gather variant 4 streams each row over its frames (two wavefronts
    load rows two frames ahead, two assemble and store), for rows that are
    16-byte multiples of at most 16 KiB; other rows of the same launch are
    gathered as by variant 0.  Buffers of odd length, with and without
    masks, batched and plain, against the oracle."""
    host = [synth.make_clip(seed, N, H, W, C=C, n_obj=2, cut_at=N // 2, lattice=8)
            for seed, N, H, W, C, Wt, k in STREAMED]
    want = [orc.retarget(f, sp[5], sp[6]) for f, sp in zip(host, STREAMED)]
    ctx.kernel_variants(0, 0, 0, 4, 0)
    try:
        clips = [dict(frames=dev(f), target_width=sp[5], seams_per_iter=sp[6], want_masks=want_masks)
                 for f, sp in zip(host, STREAMED)]
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
        plain = [ctx.retarget(dev(f), sp[5], sp[6], want_masks=want_masks) for f, sp in zip(host, STREAMED[:3])]
        torch.cuda.synchronize()
    finally:
        ctx.kernel_variants()
    for c, w in zip(clips, want):
        assert np.array_equal(c["out"].cpu().numpy(), w["out"])
        if want_masks:
            assert np.array_equal(masks_u16(c["masks"]), w["masks"])
    for g, w in zip(plain, want):
        assert np.array_equal(g["out"].cpu().numpy(), w["out"])
        if want_masks:
            assert np.array_equal(masks_u16(g["masks"]), w["masks"])


def test_kernel_variants_refused(ctx):
    from paper_1903_03180_amd import scpl
    for v in ((-1, 0, 0, 0, 0), (7, 0, 0, 0, 0), (0, -1, 0, 0, 0), (0, 3, 0, 0, 0), (0, 0, -1, 0, 0),
              (0, 0, 3, 0, 0), (0, 0, 0, -1, 0), (0, 0, 0, 5, 0), (0, 0, 0, 0, -1), (0, 0, 0, 0, 3)):
        with pytest.raises(scpl.ScplError):
            ctx.kernel_variants(*v)


def test_autotune_batch_keeps_results(orc):
    """The batch autotuner times whole batched retargets under every
    candidate configuration (writing the outputs each time) and keeps the
    fastest; the outputs it leaves, and a batched call afterwards, are the
    oracle's."""
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    try:
        frames = [synth.make_clip(670 + i, 10, 48, 200 + 40 * i, C=1, n_obj=3, cut_at=5, lattice=8) for i in range(4)]
        clips = [dict(frames=dev(f), target_width=(3 * f.shape[2]) // 4, seams_per_iter=8, want_masks=True)
                 for f in frames]
        choice = c.autotune_batch(clips, reps=1)
        torch.cuda.synchronize()
        assert choice["streams"] in (2, 3, 4) and choice["ms"] > 0
        assert 0 <= choice["update_variant"] < 7 and 0 <= choice["refresh_variant"] < 3
        assert 0 <= choice["borg_variant"] < 3 and 0 <= choice["gather_variant"] < 5
        assert 0 <= choice["fuse_variant"] < 3
        assert choice["batch_mode"] in (0, 1) and choice["persist_workgroups"] > 0
        for cl, f in zip(clips, frames):
            want = orc.retarget(f, cl["target_width"], 8)
            assert np.array_equal(cl["out"].cpu().numpy(), want["out"])
            assert np.array_equal(masks_u16(cl["masks"]), want["masks"])
        again = [dict(frames=cl["frames"], target_width=cl["target_width"], seams_per_iter=8) for cl in clips]
        c.retarget_batch(again)
        torch.cuda.synchronize()
        for a, cl in zip(again, clips):
            assert torch.equal(a["out"], cl["out"])
        c.dp_geometry(8, 16, 8, 1)
        with pytest.raises(scpl.ScplError):
            c.autotune_batch(clips, reps=1)
    finally:
        c.close()


@pytest.mark.parametrize("fuse", [1, 2])
def test_fused_band_update_uneven_and_tall(ctx, orc, fuse):
    """The fused per-band kernel on shapes with a ragged last band, one-row
    and 33-row frames, several buffers, RGB and luma, and widths over its
    1024-column compaction pass, against the oracle; and a launch it does not
    serve (more than 64 seams per iteration) falling back to two launches."""
    cases = [(synth.make_clip(680, 9, 33, 300, C=3, n_obj=3, cut_at=4, lattice=8), 220, 6),
             (synth.make_clip(681, 5, 1, 90, C=1, n_obj=2, lattice=8), 60, 4),
             (synth.make_clip(682, 6, 70, 2300, C=1, n_obj=3, cut_at=3, lattice=16), 2200, 16),
             (synth.make_clip(683, 7, 64, 120, C=1, n_obj=3, cut_at=3, lattice=8), 80, 200)]
    ctx.kernel_variants(0, 0, 0, 0, fuse)
    try:
        for f, wt, k in cases:
            compare(ctx, orc, f, wt, k)
        clips = [dict(frames=dev(f), target_width=wt, seams_per_iter=k, want_masks=True) for f, wt, k in cases[:3]]
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
    finally:
        ctx.kernel_variants()
    for c, (f, wt, k) in zip(clips, cases):
        want = orc.retarget(f, wt, k)
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(masks_u16(c["masks"]), want["masks"])


def test_batch_graph_replayed_across_calls(ctx, orc):
    """A job group replays the iteration graph of the previous call when its
    launches would be the same (same job table, shapes, geometry and kernel
    variants; the kernels read the job table when they run).  Batches of
    the same shapes with other frames, one after another, and the first
    again, each against the oracle; then a batch of other shapes."""
    shapes = [(9, 40, 120, 3, 90, 6), (12, 33, 150, 1, 110, 4), (7, 50, 96, 1, 70, 8), (10, 24, 200, 3, 150, 5)]

    def batch(seed0, shp):
        host = [synth.make_clip(seed0 + q, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
                for q, (N, H, W, C, Wt, k) in enumerate(shp)]
        clips = [dict(frames=dev(f), target_width=Wt, seams_per_iter=k, want_masks=True)
                 for f, (N, H, W, C, Wt, k) in zip(host, shp)]
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
        for c, f, (N, H, W, C, Wt, k) in zip(clips, host, shp):
            want = orc.retarget(f, Wt, k)
            assert np.array_equal(c["out"].cpu().numpy(), want["out"])
            assert np.array_equal(masks_u16(c["masks"]), want["masks"])

    for seed0 in (720, 730, 720):
        batch(seed0, shapes)
    batch(740, [(8, 30, 100, 1, 80, 3), (6, 28, 64, 3, 50, 2)])
