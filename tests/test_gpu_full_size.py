"""Every iteration of the full-size workloads against the oracle.

tests/golden/full_size_sha256.json holds SHA-256 digests of the CPU
oracle's whole retarget of each workload (output frames, masks, buffer ids
and the (buffer, W_r, P_eff, k_iter) record of every iteration), written by
tests/golden/make_full_size.py, which calls only the oracle.  Here the HIP
library retargets the same seeded clips, in the launch configurations the
benchmark times, and the digests of its results must be the oracle's:

  * the 1080p clip (seed 2) on the plain path, default and column-split DP;
  * the 16 clips of the 1080p batch in one batched call (three job groups,
    the column-split DP (4,16,8) with 256 rows x 384 columns that the
    benchmark's autotuner picks), and each of the first four alone;
  * the 4K clip at alpha 3/20, 1/5 and 1/4 on the plain path, and the three
    in one batched call;
  * the first 16 clips of the uneven mix in one batched call;
  * the 1080p batch, the three 4K runs and the mix also in the persistent
    launch (SCPL_BATCH_PERSISTENT), on a stream of their own.
"""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1903_03180_amd import synth  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_sha256.json")


def goldens():
    with open(GOLDEN) as f:
        return json.load(f)["workloads"]


G = goldens() if os.path.exists(GOLDEN) else {}


def need(*names):
    missing = [n for n in names if n not in G]
    if missing:
        pytest.fail(f"no oracle digest for {missing}: run tests/golden/make_full_size.py")
    return [G[n] for n in names]


def frames_of(rec):
    if rec["kind"] == "1080p":
        return synth.clip_1080p(rec["seed"])
    if rec["kind"] == "4k":
        return synth.clip_4k(rec["seed"])
    return synth.clip_from_spec(synth.ClipSpec(rec["seed"], rec["N"], rec["H"], rec["W"], rec["Wt"]))


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digests(out, masks, bid, log):
    return dict(out=sha(out.cpu().numpy()), masks=sha(masks.cpu().numpy().view(np.uint16)),
                buffer_id=sha(bid.cpu().numpy()), log=sha(np.ascontiguousarray(log, dtype=np.int32)))


def check(name, got, log):
    want = G[name]
    d = digests(got["out"], got["masks"], got["buffer_id"], log)
    bufs = np.bincount(got["buffer_id"].cpu().numpy()).tolist()
    assert bufs == want["buffers"], (name, bufs)
    assert len(log) == want["iterations"], (name, len(log))
    for key in ("buffer_id", "log", "masks", "out"):
        assert d[key] == want["sha256"][key], (name, key)


@pytest.fixture(scope="module")
def ctx():
    from paper_1903_03180_amd import scpl
    c = scpl.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_plain(ctx, rec, frames):
    res = ctx.retarget(frames, rec["Wt"], rec["k"], alpha_num=rec["anum"], alpha_den=rec["aden"])
    torch.cuda.synchronize()
    return res, ctx.last_log()


def run_batch(ctx, recs, frames, nstreams=3, persistent=False):
    from paper_1903_03180_amd import scpl
    clips = [dict(frames=f, target_width=r["Wt"], seams_per_iter=r["k"], alpha_num=r["anum"],
                  alpha_den=r["aden"], want_masks=True) for r, f in zip(recs, frames)]
    ctx.batch_streams(nstreams)
    if persistent:
        ctx.batch_mode(scpl.SCPL_BATCH_PERSISTENT)
    try:
        if persistent:
            torch.cuda.synchronize()
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                ctx.retarget_batch(clips, stream=s)
            s.synchronize()
        else:
            ctx.retarget_batch(clips)
            torch.cuda.synchronize()
    finally:
        ctx.batch_streams(3)
        ctx.batch_mode(scpl.SCPL_BATCH_GROUPS)
    log = ctx.last_log()
    # the batched log holds the clips' records in order
    out, at = [], 0
    for r, c in zip(recs, clips):
        n = G[r["_name"]]["iterations"]
        out.append((c, log[at:at + n]))
        at += n
    assert at == len(log)
    return out


@pytest.mark.parametrize("geom,variants", [(None, None), ((4, 16, 8, 1, 256, 384), None),
                                           ((8, 16, 8, 1, 0, 0), (1, 0, 1, 1, 1)), (None, (0, 0, 0, 0, 2))])
def test_1080p_clip_every_iteration(ctx, geom, variants):
    (rec,) = need("clip1080p_s2")
    d = dev(frames_of(rec["recipe"]))
    if geom:
        ctx.dp_geometry(*geom[:4])
        ctx.dp_chunking(*geom[4:])
    if variants:
        ctx.kernel_variants(*variants)
    try:
        res, log = run_plain(ctx, rec["recipe"], d)
    finally:
        ctx.dp_geometry(0)
        ctx.kernel_variants()
    check("clip1080p_s2", res, log)


def test_1080p_batch_as_benchmarked_every_iteration(ctx):
    """The benchmark's 16 clips of 1080p in one batched call."""
    names = [f"clip1080p_s{s}" for s in range(2000, 2016)]
    recs = need(*names)
    rr = [dict(r["recipe"], _name=n) for n, r in zip(names, recs)]
    frames = [dev(frames_of(r)) for r in rr]
    ctx.dp_geometry(4, 16, 8, 1)
    ctx.dp_chunking(256, 384)
    try:
        res = run_batch(ctx, rr, frames)
    finally:
        ctx.dp_geometry(0)
    for n, (c, log) in zip(names, res):
        check(n, c, log)
    # and with the fused per-band kernel and the other kernel variants
    ctx.kernel_variants(1, 0, 0, 1, 1)
    try:
        res = run_batch(ctx, rr, frames)
    finally:
        ctx.kernel_variants()
    for n, (c, log) in zip(names, res):
        check(n, c, log)
    # and in the persistent launch
    for n, (c, log) in zip(names, run_batch(ctx, rr, frames, persistent=True)):
        check(n, c, log)
    # the same clips alone on the plain path (default geometry)
    for n, r, f in list(zip(names, rr, frames))[:4]:
        got, log = run_plain(ctx, r, f)
        check(n, got, log)


def test_4k_clip_alpha_sweep_every_iteration(ctx):
    names = [f"clip4k_s3_a{a}_{d}" for a, d in ((3, 20), (1, 5), (1, 4))]
    recs = need(*names)
    rr = [dict(r["recipe"], _name=n) for n, r in zip(names, recs)]
    d = dev(frames_of(rr[0]))
    for n, r in zip(names, rr):
        got, log = run_plain(ctx, r, d)
        check(n, got, log)
    for n, (c, log) in zip(names, run_batch(ctx, rr, [d, d, d])):
        check(n, c, log)
    for n, (c, log) in zip(names, run_batch(ctx, rr, [d, d, d], persistent=True)):
        check(n, c, log)


def test_uneven_mix_batch_every_iteration(ctx):
    names = sorted((n for n in G if n.startswith("mix_")), key=lambda n: int(n[4:]))
    assert len(names) >= 16
    rr = [dict(G[n]["recipe"], _name=n) for n in names]
    frames = [dev(frames_of(r)) for r in rr]
    for n, (c, log) in zip(names, run_batch(ctx, rr, frames)):
        check(n, c, log)
    for n, (c, log) in zip(names, run_batch(ctx, rr, frames, persistent=True)):
        check(n, c, log)
