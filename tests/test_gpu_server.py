"""Request server (continuous batching): every request's result is
bit-identical alone, inside a mix of uneven clips submitted while others
are running, and to the oracle; a request is done when its own buffers are,
not when its batch is; admission follows the device-memory budget."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# uneven sizes, aspect ratios, lengths, luma and RGB, gradient and motion
MIX = [
    dict(seed=900, N=14, H=40, W=90, C=3, Wt=67, k=4),
    dict(seed=901, N=30, H=24, W=120, C=1, Wt=90, k=16),
    dict(seed=902, N=6, H=64, W=64, C=1, Wt=48, k=8, energy_mode=0),
    dict(seed=903, N=20, H=36, W=180, C=3, Wt=135, k=2, alpha_num=3, alpha_den=20),
    dict(seed=904, N=9, H=90, W=50, C=1, Wt=37, k=1000),
    dict(seed=905, N=25, H=18, W=256, C=1, Wt=192, k=16, use_buffer=0),
    dict(seed=906, N=11, H=48, W=72, C=3, Wt=54, k=6, max_buffer=4),
]


def make(spec):
    N, H, W, C = spec["N"], spec["H"], spec["W"], spec["C"]
    return synth.make_clip(spec["seed"], N, H, W, C=C, n_obj=3, cut_at=N // 2, lattice=8)


def kwargs(spec):
    return {k: spec[k] for k in ("energy_mode", "use_buffer", "alpha_num", "alpha_den", "max_buffer") if k in spec}


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


def test_server_results_alone_and_in_the_mix(ctx, orc):
    from paper_1903_03180_amd import scpl
    frames = [make(s) for s in MIX]
    solo = [ctx.retarget(dev(f), s["Wt"], s["k"], **kwargs(s)) for f, s in zip(frames, MIX)]
    torch.cuda.synchronize()
    srv = scpl.Server(0, lanes=3, max_batch=2)
    try:
        tickets = []
        for rep in range(2):  # every clip twice: more requests than lanes
            for f, s in zip(frames, MIX):
                clip = dict(frames=dev(f), target_width=s["Wt"], seams_per_iter=s["k"], want_masks=True, **kwargs(s))
                torch.cuda.synchronize()
                tickets.append(srv.submit(clip))
                time.sleep(0.001)  # later requests arrive while earlier ones run
        for q, t in enumerate(tickets):
            r = srv.wait(t)
            a = solo[q % len(MIX)]
            assert torch.equal(r["out"], a["out"])
            assert torch.equal(r["masks"], a["masks"])
            assert torch.equal(r["buffer_id"], a["buffer_id"])
            qms, tms = srv.times(t)
            assert 0 <= qms <= tms
            srv.release(t)
    finally:
        srv.close()
    # and the solo results are the oracle's
    for f, s, a in zip(frames, MIX, solo):
        okw = dict(mode=s.get("energy_mode", 1), use_buffer=s.get("use_buffer", 1), anum=s.get("alpha_num", 1),
                   aden=s.get("alpha_den", 5), max_buffer=s.get("max_buffer", 0))
        want = orc.retarget(f, s["Wt"], s["k"], **okw)
        assert np.array_equal(a["out"].cpu().numpy(), want["out"])
        assert np.array_equal(a["masks"].cpu().numpy().view(np.uint16), want["masks"])
        assert np.array_equal(a["buffer_id"].cpu().numpy(), want["buffer_id"])


def test_small_request_done_before_its_batch(ctx, orc):
    """One lane: a long request (one seam per iteration) and a small one
    taken in the same batch.  The small request is done as soon as its own
    buffers are carved and gathered, well before the long one; both results
    are the plain path's, the small one also the oracle's."""
    from paper_1903_03180_amd import scpl
    big = synth.make_clip(911, 8, 1080, 1920, C=1, n_obj=4, lattice=32)
    small = make(MIX[0])
    dbig, dsmall = dev(big), dev(small)
    solo_big = ctx.retarget(dbig, 1420, 1)
    torch.cuda.synchronize()
    srv = scpl.Server(0, lanes=1, max_batch=4)
    try:
        # a first request keeps the lane busy (a few hundred iterations), so
        # that the next two are queued together and taken as one batch; the
        # pause lets the lane take the first one alone before they arrive
        first = dev(synth.make_clip(912, 6, 540, 960, C=1, n_obj=3, lattice=32))
        torch.cuda.synchronize()
        t0 = srv.submit(dict(frames=first, target_width=660, seams_per_iter=1))
        time.sleep(0.02)
        tb = srv.submit(dict(frames=dbig, target_width=1420, seams_per_iter=1, want_masks=True))
        ts = srv.submit(dict(frames=dsmall, target_width=MIX[0]["Wt"], seams_per_iter=MIX[0]["k"], want_masks=True))
        assert not srv.poll(t0)[0]  # still running: the two were queued behind it
        srv.wait(t0)
        rs = srv.wait(ts)
        done_big, _ = srv.poll(tb)
        qs, tot_s = srv.times(ts)
        rb = srv.wait(tb)
        qb, tot_b = srv.times(tb)
    finally:
        srv.close()
    assert not done_big  # the small request was done while the long one carved on
    assert tot_s - qs + 20.0 < tot_b - qb  # its time in the lane, against the long one's
    want = orc.retarget(small, MIX[0]["Wt"], MIX[0]["k"])
    assert np.array_equal(rs["out"].cpu().numpy(), want["out"])
    assert np.array_equal(rs["masks"].cpu().numpy().view(np.uint16), want["masks"])
    assert torch.equal(rb["out"], solo_big["out"]) and torch.equal(rb["masks"], solo_big["masks"])


@pytest.mark.skip(reason="iteration-level joining (a live job table per lane) was taken out after the benchmark's serving run with it faulted the GPU (memory aperture violation) without a cause found in the code; the server runs each admitted batch to completion again")
def test_small_request_joins_and_leaves_before_a_large_one(ctx, orc):
    """One lane: a long request (one seam per iteration, 500 iterations)
    starts carving; a small one submitted while it runs joins the same
    table between iterations and is done well before the long one.  Both
    results are the plain path's, the small one also the oracle's."""
    from paper_1903_03180_amd import scpl
    big = synth.make_clip(910, 8, 1080, 1920, C=1, n_obj=4, lattice=32)
    small = make(MIX[0])
    dbig, dsmall = dev(big), dev(small)
    solo_big = ctx.retarget(dbig, 1420, 1)
    torch.cuda.synchronize()
    srv = scpl.Server(0, lanes=1, max_batch=4)
    try:
        tb = srv.submit(dict(frames=dbig, target_width=1420, seams_per_iter=1, want_masks=True))
        time.sleep(0.02)
        ts = srv.submit(dict(frames=dsmall, target_width=MIX[0]["Wt"], seams_per_iter=MIX[0]["k"], want_masks=True))
        rs = srv.wait(ts)
        done_big, _ = srv.poll(tb)
        _, tot_s = srv.times(ts)
        rb = srv.wait(tb)
        _, tot_b = srv.times(tb)
    finally:
        srv.close()
    assert not done_big  # the small request finished while the long one carved on
    assert tot_s + 20.0 < tot_b
    want = orc.retarget(small, MIX[0]["Wt"], MIX[0]["k"])
    assert np.array_equal(rs["out"].cpu().numpy(), want["out"])
    assert np.array_equal(rs["masks"].cpu().numpy().view(np.uint16), want["masks"])
    assert torch.equal(rb["out"], solo_big["out"]) and torch.equal(rb["masks"], solo_big["masks"])


def test_failing_request_fails_alone(ctx):
    """A request the batched path refuses (masks asked for a clip carved in
    both dimensions) reports its error; the requests around it in the same
    lane are unaffected and bit-identical to their plain results."""
    from paper_1903_03180_amd import scpl
    frames = [make(s) for s in MIX[:3]]
    solo = [ctx.retarget(dev(f), s["Wt"], s["k"], **kwargs(s)) for f, s in zip(frames, MIX)]
    torch.cuda.synchronize()
    bad = make(MIX[3])
    srv = scpl.Server(0, lanes=1, max_batch=8)
    try:
        ts = []
        for i, (f, s) in enumerate(zip(frames, MIX)):
            ts.append(srv.submit(dict(frames=dev(f), target_width=s["Wt"], seams_per_iter=s["k"], want_masks=True,
                                      **kwargs(s))))
            if i == 1:
                tbad = srv.submit(dict(frames=dev(bad), target_width=MIX[3]["Wt"], target_height=30,
                                       seams_per_iter=4, want_masks=True))
        with pytest.raises(scpl.ScplError) as e:
            srv.wait(tbad)
        assert e.value.status == scpl.SCPL_ERR_INVALID_ARG
        for t, a in zip(ts, solo):
            r = srv.wait(t)
            assert torch.equal(r["out"], a["out"]) and torch.equal(r["masks"], a["masks"])
            assert torch.equal(r["buffer_id"], a["buffer_id"])
    finally:
        srv.close()


def test_server_admission_by_budget(ctx):
    from paper_1903_03180_amd import scpl
    spec = MIX[0]
    f = make(spec)
    p = scpl.params_for(dev(f), spec["Wt"], spec["k"])
    need = scpl.Server.footprint(p)
    assert need > 0
    # a budget below one request: refused at submission, nothing queued
    srv = scpl.Server(0, lanes=2, max_batch=4, hbm_budget=need - 1)
    try:
        with pytest.raises(scpl.ScplError) as ei:
            srv.submit(dict(frames=dev(f), target_width=spec["Wt"], seams_per_iter=spec["k"]))
        assert ei.value.status == scpl.SCPL_ERR_CAPACITY
    finally:
        srv.close()
    # room for one request at a time: requests queue and all complete
    solo = ctx.retarget(dev(f), spec["Wt"], spec["k"])
    srv = scpl.Server(0, lanes=3, max_batch=4, hbm_budget=need + need // 2)
    try:
        ts = [srv.submit(dict(frames=dev(f), target_width=spec["Wt"], seams_per_iter=spec["k"])) for _ in range(4)]
        spans = []
        for t in ts:
            r = srv.wait(t)
            assert torch.equal(r["out"], solo["out"])
            spans.append(srv.times(t))
        # one at a time: the later requests waited in the queue
        assert max(q for q, _ in spans) > 0
    finally:
        srv.close()


def test_server_rejects_invalid_requests():
    from paper_1903_03180_amd import scpl
    srv = scpl.Server(0, lanes=1, max_batch=1)
    try:
        f = dev(make(MIX[1]))
        with pytest.raises(scpl.ScplError):
            srv.submit(dict(frames=f, target_width=0, seams_per_iter=4))
        with pytest.raises(scpl.ScplError):
            srv.poll(12345)
    finally:
        srv.close()


def test_whole_batch_completion_results(ctx):
    """With whole_batch, every request of a batch completes with its batch
    (the early-completion path switched off): the results are still the ones
    each clip gets alone."""
    from paper_1903_03180_amd import scpl
    frames = [make(s) for s in MIX]
    solo = [ctx.retarget(dev(f), s["Wt"], s["k"], **kwargs(s)) for f, s in zip(frames, MIX)]
    torch.cuda.synchronize()
    srv = scpl.Server(0, lanes=1, max_batch=len(MIX), whole_batch=True)
    try:
        clips = [dict(frames=dev(f), target_width=s["Wt"], seams_per_iter=s["k"], want_masks=True, **kwargs(s))
                 for f, s in zip(frames, MIX)]
        torch.cuda.synchronize()
        tickets = [srv.submit(c) for c in clips]
        results = [srv.wait(t) for t in tickets]
        for r, a in zip(results, solo):
            assert torch.equal(r["out"], a["out"])
            assert torch.equal(r["masks"], a["masks"])
            assert torch.equal(r["buffer_id"], a["buffer_id"])
        for t in tickets:
            srv.release(t)
    finally:
        srv.close()
