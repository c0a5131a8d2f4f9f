"""The persistent launch of the batched path (SCPL_BATCH_PERSISTENT) against
the oracle: one launch runs every iteration of every buffer of the batch,
its workgroups taking work items (DP chunks, bands, selections, refresh
rows) from a ring on the device.  Output pixels, masks, buffer ids and the
per-iteration record must equal the oracle's, on a caller stream (the launch
captured as a graph) and on the default stream (launched directly), for
uneven clips: ragged last bands, one-row and one-column frames, more than 64
seams per iteration, the uncapped case, both energies, seam memorisation,
and width-and-height retargeting."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    c.batch_mode(scpl.SCPL_BATCH_PERSISTENT)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def masks_u16(t):
    return t.cpu().numpy().view(np.uint16)


def oracle_kw(c):
    return dict(mode=c.get("energy_mode", 1), use_buffer=c.get("use_buffer", 1), anum=c.get("alpha_num", 1),
                aden=c.get("alpha_den", 5), max_buffer=c.get("max_buffer", 0), memo_period=c.get("memo_period", 0))


# (seed, N, H, W, C, Wt, k, extra parameters)
MIX = [
    (600, 12, 40, 90, 3, 70, 4, {}),
    (601, 9, 65, 33, 1, 24, 16, {}),
    (602, 15, 20, 200, 1, 150, 2, dict(alpha_num=3, alpha_den=20)),
    (603, 8, 33, 300, 3, 220, 6, dict(energy_mode=0)),              # ragged last band (33 rows)
    (604, 5, 1, 90, 1, 60, 4, {}),                                  # one row
    (605, 6, 70, 400, 1, 300, 200, {}),                             # more than 64 seams per iteration
    (606, 7, 24, 150, 1, 100, 1000, dict(use_buffer=0)),            # uncapped: one seam per parent
    (607, 16, 30, 80, 3, 60, 4, dict(memo_period=2, max_buffer=2)),  # seam memorisation
    (608, 10, 97, 1000, 1, 750, 16, dict(max_buffer=3)),            # three 384-column DP parts, four 256-row chunks
]


def make(spec):
    seed, N, H, W, C, Wt, k, kw = spec
    f = synth.make_clip(seed, N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)
    return f, dict(target_width=Wt, seams_per_iter=k, **kw)


def run_and_check(ctx, orc, specs, stream):
    host, clips = [], []
    for sp in specs:
        f, c = make(sp)
        host.append(f)
        c["frames"] = dev(f)
        c["want_masks"] = True
        clips.append(c)
    torch.cuda.synchronize()
    if stream is not None:
        with torch.cuda.stream(stream):
            ctx.retarget_batch(clips, stream=stream)
        stream.synchronize()
    else:
        ctx.retarget_batch(clips)
        torch.cuda.synchronize()
    log = ctx.last_log()
    at = 0
    for c, f in zip(clips, host):
        want = orc.retarget(f, c["target_width"], c["seams_per_iter"], **oracle_kw(c))
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])
        assert np.array_equal(masks_u16(c["masks"]), want["masks"])
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        n = len(want["log"])
        assert np.array_equal(log[at:at + n], want["log"])
        at += n
    assert at == len(log)


@pytest.mark.parametrize("on_stream", [True, False])
def test_persistent_batch_equals_oracle(ctx, orc, on_stream):
    run_and_check(ctx, orc, MIX, torch.cuda.Stream() if on_stream else None)


def test_xcd_local_mode_found(ctx):
    """The probe at context creation finds the MI355X's eight XCDs, so the
    tests above ran the XCD-local kernel."""
    assert ctx.device_xcds() == 8


@pytest.mark.skip(reason="the one-ring agent-scope persistent kernel is switched off: a run of this test faulted the "
                         "GPU (illegal address) after the XCD-local tests had passed, with no cause found in its code")
def test_agent_mode_equals_oracle(ctx, orc):
    """The one-ring kernel with agent-scope ordering (the fallback when the
    XCD of a workgroup cannot be trusted)."""
    from paper_1903_03180_amd import scpl
    ctx.batch_mode(scpl.SCPL_BATCH_PERSISTENT_AGENT)
    try:
        run_and_check(ctx, orc, MIX, torch.cuda.Stream())
    finally:
        ctx.batch_mode(scpl.SCPL_BATCH_PERSISTENT)


def test_persistent_single_clips_and_repeat(ctx, orc):
    """One clip per call, twice in a row (the ring and counters are set up
    afresh by each launch)."""
    s = torch.cuda.Stream()
    for sp in (MIX[5], MIX[0], MIX[5]):
        run_and_check(ctx, orc, [sp], s)


def test_persistent_width_and_height(ctx, orc):
    specs = [(710, 9, 30, 50, 3, 40, 30), (711, 6, 44, 26, 1, 26, 33), (712, 10, 28, 40, 1, 31, 20)]
    clips, host = [], []
    for seed, N, H, W, C, Wt, Ht in specs:
        f = synth.make_clip(seed, N, H, W, C=C, n_obj=2, cut_at=N // 2, lattice=8)
        host.append((f, Wt, Ht))
        clips.append(dict(frames=dev(f), target_width=Wt, target_height=Ht, seams_per_iter=6))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.retarget_batch(clips, stream=s)
    s.synchronize()
    for c, (f, Wt, Ht) in zip(clips, host):
        want = orc.retarget_2d(f, Wt, Ht, 6)
        assert np.array_equal(c["out"].cpu().numpy(), want["out"])
        assert np.array_equal(c["buffer_id"].cpu().numpy(), want["buffer_id"])


def test_persistent_equals_groups_and_profiles(ctx, orc):
    """With event timing on, the persistent kernel runs outside a graph and
    is timed as its own kind; the results equal the job-group path's."""
    from paper_1903_03180_amd import scpl
    specs = MIX[:4]
    ctx.profile(True)
    try:
        run_and_check(ctx, orc, specs, torch.cuda.Stream())
        prof = ctx.profile_read()
    finally:
        ctx.profile(False)
    assert prof["persist"][1] == 1 and prof["persist"][0] > 0
    assert prof["dp"][1] == 0 and prof["update"][1] == 0
    st = ctx.persist_stats()
    parts = ("dp", "borg", "select", "band", "refresh")
    assert all(st[k][1] > 0 and st[k][0] > 0 for k in parts)
    assert st["wait"][1] == st["done"][1] >= sum(st[k][1] for k in parts)
    ctx.batch_mode(scpl.SCPL_BATCH_GROUPS)
    try:
        run_and_check(ctx, orc, specs, torch.cuda.Stream())
    finally:
        ctx.batch_mode(scpl.SCPL_BATCH_PERSISTENT)


def test_batch_mode_refused(ctx):
    from paper_1903_03180_amd import scpl
    for m in (-1, 3, scpl.SCPL_BATCH_PERSISTENT_AGENT):
        with pytest.raises(scpl.ScplError):
            ctx.batch_mode(m)
