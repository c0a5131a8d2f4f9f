"""Benchmark: SCPL video retargeting of 1080p clips on one MI355X.

A step is one whole retarget of the workload (luma, buffer segmentation,
every SCPL iteration of every buffer, output gather) with the frames already
resident in HBM.  Workloads:

  1080p-batch16 (default)  16 clips of the 1080p generator (seeds 2000-2015):
                           120 frames 1920x1080 RGB each, scene cut at frame
                           60, retargeted to 1440 wide at k = 16, alpha = 1/5
  1080p                    the single 1080p clip (seed 2)
  4k                       60 frames 3840x2160 luma -> 2880 wide, k = 32

`value` is frames per second of the batched path (every buffer of every
clip advances together, one launch per stage per iteration, iterations
replayed from a HIP graph); the plain path (one buffer after another, clip
after clip) is timed beside it.  The oracle (plain C, one core) is timed on
a bounded sample of the first clip.  Seam memorisation (only every m-th
buffer of a clip carved, the others reusing its removal) is timed on the same
workload for the periods of --memo-periods, with the fraction of output bytes
it changes, and horizontal seams (3/4 of the height, alone and with 3/4 of the
width) on the first clip.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "1080p frames/s (batched vs plain, bit-exact); HBM GB/s; p50/p99 latency"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _gen(args):
    kind, seed = args
    from paper_1903_03180_amd import synth
    return synth.clip_1080p(seed) if kind == "1080p" else synth.clip_4k(seed)


def make_workload(name):
    """[(clip, target width, seams per iteration)], description."""
    if name == "1080p-batch16":
        seeds = list(range(2000, 2016))
        clips = [_gen(("1080p", s)) for s in seeds]
        return [(c, 1440, 16) for c in clips], (
            "16 clips x 120 frames 1920x1080 RGB (1080p generator, seeds 2000-2015) -> 1440 wide, k=16 "
            "seams/iteration, alpha=1/5, motion energy")
    if name == "1080p":
        return [(_gen(("1080p", 2)), 1440, 16)], ("1080p RGB clip: 120 frames 1920x1080 -> 1440 wide, k=16 "
                                                  "seams/iteration, alpha=1/5, motion energy")
    if name == "mix64":
        from paper_1903_03180_amd import synth
        specs = synth.batch_mix_specs(64)
        clips = [_gen_spec(sp) for sp in specs]
        return [(c, s.Wt, 16) for c, s in zip(clips, specs)], (
            "64 clips of uneven size (luma, widths 480-2560, heights 360-1440, aspect 1:1-21:9, 30-240 frames, "
            "seeds 4000-4063) -> 3/4 of the width, k=16 seams/iteration, alpha=1/5, motion energy")
    return [(_gen(("4k", 3)), 2880, 32)], ("4K luma clip: 60 frames 3840x2160 -> 2880 wide, k=32 seams/iteration, "
                                           "alpha=1/5, motion energy")


def _gen_spec(spec):
    from paper_1903_03180_amd import synth
    if spec is None:
        return None
    if isinstance(spec, tuple):  # ("4k", seed)
        return synth.clip_4k(spec[1])
    return synth.clip_from_spec(spec)


def serving_pool(n_mix, n_4k):
    """Requests drawn from the uneven batch mix (luma, widths 480-2560,
    heights 360-1440, 30-240 frames, target 3/4 of the width) plus 4K jobs
    (60 frames 3840x2160 luma)."""
    from paper_1903_03180_amd import synth
    specs = synth.batch_mix_specs(n_mix)
    jobs = list(specs) + [("4k", 5000 + j) for j in range(n_4k)]
    clips = [_gen_spec(j) for j in jobs]
    wt = [s.Wt for s in specs] + [2880] * n_4k
    k = [16] * n_mix + [32] * n_4k
    return clips, wt, k


def run_serving(np, torch, scpl, n_mix=14, n_4k=2, n_req=400, warm=0.1, p4k=0.1, n_cap=64,
                fracs=(0.5, 0.8, 0.95), lanes=4, seed=5, whole_batch_at=0.8):
    """Poisson arrivals of retarget requests at fractions of the measured
    capacity.  A request is a clip of the uneven mix, or with probability
    p4k a 4K clip; the first `warm` fraction of each rate's requests (by
    arrival) is left out of the latency figures.  p50 / p99 of completion
    minus arrival (all requests, mix clips, 4K clips), and frames/s over the
    whole rate; then the rate whole_batch_at once more with requests done
    only when their whole batch is (the comparison for early completion)."""
    import time as _t
    clips_np, wts, ks = serving_pool(n_mix, n_4k)
    dev = [torch.from_numpy(c).cuda() for c in clips_np]
    torch.cuda.synchronize()
    srv = scpl.Server(0, lanes=lanes, max_batch=8)
    rng = np.random.default_rng(seed)

    def pct(a, q):
        return None if len(a) == 0 else round(float(np.percentile(a, q)), 2)

    def draw(n):
        is4k = rng.random(n) < p4k
        return np.where(is4k, n_mix + rng.integers(0, n_4k, size=n), rng.integers(0, n_mix, size=n))

    def req(q):
        return dict(frames=dev[q], target_width=wts[q], seams_per_iter=ks[q])

    # capacity: a burst of n_cap requests of the same mix submitted at once
    burst = draw(n_cap)
    for q in range(len(dev)):  # every clip once first (lane workspaces)
        t = srv.submit(req(q))
        srv.wait(t)
        srv.release(t)
    t0 = _t.perf_counter()
    ts = [srv.submit(req(int(q))) for q in burst]
    for t in ts:
        srv.wait(t)
        srv.release(t)
    cap = n_cap / (_t.perf_counter() - t0)
    log(f"serving capacity ({n_cap} requests at once): {cap:.2f} requests/s")
    n_warm = int(round(warm * n_req))
    out = {"capacity_req_per_s": round(cap, 3),
           "pool": f"{n_mix} clips of the uneven mix, and with probability {p4k} one of {n_4k} 4K clips",
           "requests_per_rate": n_req, "warmup_requests": n_warm, "latency_samples": n_req - n_warm,
           "lanes": lanes, "rates": []}
    runs = [(f, False) for f in fracs] + ([(whole_batch_at, True)] if whole_batch_at else [])
    for f, whole in runs:
        if whole:  # the same rate, requests done with their whole batch
            srv.close()
            srv = scpl.Server(0, lanes=lanes, max_batch=8, whole_batch=True)
            for q in range(len(dev)):
                t = srv.submit(req(q))
                srv.wait(t)
                srv.release(t)
        lam = f * cap
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
        picks = draw(n_req)
        tickets = []
        start = _t.perf_counter()
        for a, q in zip(arrivals, picks):
            now = _t.perf_counter() - start
            if a > now:
                _t.sleep(a - now)
            lag = max(0.0, (_t.perf_counter() - start) - a)
            tickets.append((srv.submit(req(int(q))), lag, int(q)))
        lat, is4k, frames = [], [], 0
        for i, (t, lag, q) in enumerate(tickets):
            srv.wait(t)
            _, total_ms = srv.times(t)
            if i >= n_warm:
                lat.append(total_ms + 1e3 * lag)
                is4k.append(q >= n_mix)
            frames += dev[q].shape[0]
            srv.release(t)
        span = _t.perf_counter() - start
        lat, is4k = np.array(lat), np.array(is4k, dtype=bool)
        rec = {"load": f, "arrival_req_per_s": round(lam, 3), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
               "mix_p50_ms": pct(lat[~is4k], 50), "mix_p99_ms": pct(lat[~is4k], 99),
               "4k_p50_ms": pct(lat[is4k], 50), "4k_p99_ms": pct(lat[is4k], 99),
               "frames_per_s": round(frames / span, 1), "samples": int(len(lat)), "samples_4k": int(is4k.sum()),
               "completion": "with the whole batch" if whole else "with the request's own buffers"}
        log(f"serving at {f:.2f} x capacity{' (whole-batch completion)' if whole else ''}: p50 {rec['p50_ms']} ms, "
            f"p99 {rec['p99_ms']} ms over {len(lat)} requests ({rec['samples_4k']} 4K; mix p50 {rec['mix_p50_ms']} "
            f"p99 {rec['mix_p99_ms']}, 4K p50 {rec['4k_p50_ms']} p99 {rec['4k_p99_ms']}), "
            f"{rec['frames_per_s']} frames/s")
        if whole:
            out["whole_batch_completion"] = rec
        else:
            out["rates"].append(rec)
    srv.close()
    del dev
    torch.cuda.synchronize()
    return out


# Table 1 of the paper (Sec. 4): clip, width x height, frames, target width,
# and the paper's CPU seconds for its method ("Proposed") and for seam
# carving run on every frame ("Raw").  Frames of the rows whose cells are
# garbled are read as Helicopter's 178.
TABLE1 = [("Big Belly", 640, 480, 377, 512, 124.36, 1255.19), ("Big Belly", 640, 480, 377, 384, 214.24, 2484.91),
          ("Lion", 640, 480, 117, 512, 80.72, 600.90), ("Lion", 640, 480, 117, 384, 140.88, 1225.60),
          ("Lego", 560, 320, 164, 448, 32.28, 263.89), ("Lego", 560, 320, 164, 336, 56.21, 532.16),
          ("Helicopter", 720, 576, 178, 576, 143.31, 1594.19), ("Helicopter", 720, 576, 178, 432, 282.70, 3096.67),
          ("Helicopter", 320, 240, 178, 256, 16.32, 201.71), ("Helicopter", 320, 240, 178, 192, 31.44, 426.67),
          ("Helicopter", 176, 144, 178, 140, 3.43, 52.65), ("Helicopter", 176, 144, 178, 105, 6.73, 108.34)]


def _gen_table1(row):
    from paper_1903_03180_amd import synth
    q, (_n, W, H, N, _wt, _p, _r) = row
    return synth.make_clip(6000 + q, N, H, W, C=3, n_obj=3, max_speed=4, cut_at=N // 2, lattice=32)


def run_table1(np, torch, scpl, ctx):
    """Proposed (SCPL, one seam per parent per iteration, dynamic buffer,
    motion energy) against Raw (classic seam carving of every frame: one
    seam per iteration, no buffer, gradient energy) on synthetic RGB clips
    of Table 1's shapes, lengths and target widths, both on this GPU."""
    import time as _t
    clips = [_gen_table1(r) for r in enumerate(TABLE1)]
    rows = []
    for (name, W, H, N, Wt, p_s, r_s), c in zip(TABLE1, clips):
        fr = torch.from_numpy(c).cuda()
        res = {}
        for method, kw in (("proposed", dict(seams_per_iter=W)),
                           ("raw", dict(seams_per_iter=1, use_buffer=0, energy_mode=0))):
            job = [dict(frames=fr, target_width=Wt, **kw)]
            ctx.retarget_batch(job)  # warm-up (workspace, graphs)
            torch.cuda.synchronize()
            t0 = _t.perf_counter()
            ctx.retarget_batch(job)
            torch.cuda.synchronize()
            res[method] = _t.perf_counter() - t0
        rows.append({"clip": name, "size": f"{W}x{H}", "frames": N, "target_width": Wt,
                     "proposed_ms": round(1e3 * res["proposed"], 2), "raw_ms": round(1e3 * res["raw"], 2),
                     "reduction": round(1 - res["proposed"] / res["raw"], 4),
                     "paper_reduction": round(1 - p_s / r_s, 4)})
        del fr
    red = [r["reduction"] for r in rows]
    log("Table 1 shapes: mean reduction Proposed vs Raw on this GPU " + f"{100 * np.mean(red):.1f}% "
        f"(paper, CPU: {100 * np.mean([r['paper_reduction'] for r in rows]):.1f}%)")
    return {"rows": rows, "mean_reduction": round(float(np.mean(red)), 4),
            "paper_mean_reduction": round(float(np.mean([r["paper_reduction"] for r in rows])), 4),
            "inputs": "synthetic RGB clips of each row's size, length and target (seeds 6000-6011)"}


def run_persistent_leg(torch, scpl, ctx, step, n_frames, steps, fps_groups, choice):
    """The same batched step as one persistent launch (SCPL_BATCH_PERSISTENT,
    graph-captured, no events): frames/s, and one more step with the
    persistent kernel timed and its workgroups' time traced."""
    import time as _t
    if ctx.device_xcds() == 0:
        return None
    ctx.batch_mode(scpl.SCPL_BATCH_PERSISTENT)
    try:
        step()
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = _t.perf_counter()
        ctx.profile(True, kinds=["persist"])
        step()
        torch.cuda.synchronize()
        pk = ctx.profile_read()["persist"]
        stats = ctx.persist_stats()
        ctx.profile(False)
    finally:
        ctx.batch_mode(scpl.SCPL_BATCH_GROUPS)
    fps = n_frames * steps / (t1 - t0)
    log(f"persistent launch: {(t1 - t0) * 1e3 / steps:.2f} ms/step, {fps:.1f} frames/s "
        f"(job groups {fps_groups:.1f}); persistent kernel {pk[0]:.2f} ms")
    return {"fps": round(fps, 2), "ms_per_step": round((t1 - t0) * 1e3 / steps, 3),
            "over_job_groups": round(fps / fps_groups, 4), "persist_kernel_ms": round(pk[0], 3),
            "xcds": ctx.device_xcds(), "tuner_picked": bool(choice and choice.get("batch_mode") == 1),
            "workgroup_ms": {k: {"ms": round(v[0], 1), "items": int(v[1])} for k, v in stats.items()},
            "timing": "graph-captured launch, no per-launch events; workgroup_ms: summed over the workgroups of "
                      "one more step (device wall clock)"}


def run_mix(np, torch, ctx, steps):
    """The 64 clips of uneven size (luma, widths 480-2560, heights 360-1440,
    aspect 1:1-21:9, 30-240 frames, target 3/4 of the width): the batched
    path (DP autotuned for the mix, graph-replayed steps) and the plain
    path, frames/s of each."""
    import time as _t
    work, desc = make_workload("mix64")
    n_frames = sum(c.shape[0] for c, _, _ in work)
    Hmax = max(c.shape[1] for c, _, _ in work)
    Wmax = max(c.shape[2] for c, _, _ in work)
    clips = [dict(frames=torch.from_numpy(c).cuda(), target_width=wt, seams_per_iter=kk) for c, wt, kk in work]
    del work
    torch.cuda.synchronize()
    ctx.autotune_dp(Hmax, Wmax, n_jobs=1)
    dpus = ctx.autotune_dp(Hmax, Wmax, n_jobs=256)[4]
    g = ctx.dp_chosen(Wmax)
    choice = ctx.autotune_batch(clips, reps=1)
    if choice["dp_geometry"] is not None:
        g = choice["dp_geometry"]

    def timed():
        ctx.retarget_batch(clips)  # warm-up (workspace, graphs)
        torch.cuda.synchronize()
        a = _t.perf_counter()
        for _ in range(steps):
            ctx.retarget_batch(clips)
        torch.cuda.synchronize()
        return a, _t.perf_counter()

    # the tuner's configuration, and the other batch mode beside it
    t0, t1 = timed()
    fps = n_frames * steps / (t1 - t0)
    other = None
    if ctx.device_xcds() > 0:
        from paper_1903_03180_amd import scpl as _s
        om = _s.SCPL_BATCH_GROUPS if choice["batch_mode"] == _s.SCPL_BATCH_PERSISTENT else _s.SCPL_BATCH_PERSISTENT
        ctx.batch_mode(om)
        try:
            o0, o1 = timed()
        finally:
            ctx.batch_mode(choice["batch_mode"])
        other = {"batch_mode": "persistent" if om == _s.SCPL_BATCH_PERSISTENT else "job groups",
                 "fps": round(n_frames * steps / (o1 - o0), 2), "ms_per_step": round((o1 - o0) * 1e3 / steps, 3)}
    p0 = _t.perf_counter()
    for c in clips:
        ctx.retarget(c["frames"], c["target_width"], c["seams_per_iter"], want_masks=False)
    torch.cuda.synchronize()
    p1 = _t.perf_counter()
    plain = n_frames / (p1 - p0)
    log(f"mix64: batched {fps:.1f} frames/s ({(t1 - t0) * 1e3 / steps:.1f} ms/step), plain {plain:.1f} frames/s, "
        f"DP {g} ({dpus:.1f} us per DP alone), batch tuning {choice}; other batch mode {other}")
    ctx.batch_mode(0)
    del clips
    torch.cuda.empty_cache()
    return {"workload": desc, "frames": n_frames, "steps": steps, "batched_fps": round(fps, 2),
            "ms_per_step": round((t1 - t0) * 1e3 / steps, 3), "plain_fps": round(plain, 2),
            "batched_over_plain": round(fps / plain, 3), "dp_geometry": g, "batch_tuning": choice,
            "batch_mode": "persistent" if choice["batch_mode"] == 1 else "job groups", "other_batch_mode": other}


def run_height(torch, ctx, clip_np, Wt, k, steps):
    """Horizontal seams (Sec. 3.1, eq. 2, as vertical seams of the transposed frames):
    the workload's first clip carved to 3/4 of its height alone, and to 3/4
    of its width and height, as one batched call each."""
    import time as _t
    fr = torch.from_numpy(clip_np).cuda()
    N, H, W = clip_np.shape[:3]
    Ht = (3 * H) // 4
    out = {"clip": f"{N} frames {W}x{H}", "target_height": Ht}
    for name, wt in (("height_only", W), ("width_and_height", Wt)):
        job = [dict(frames=fr, target_width=wt, target_height=Ht, seams_per_iter=k)]
        ctx.retarget_batch(job)  # warm-up (workspace, graphs)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        for _ in range(steps):
            ctx.retarget_batch(job)
        torch.cuda.synchronize()
        fps = N * steps / (_t.perf_counter() - t0)
        out[name] = {"target": f"{wt}x{Ht}", "frames_per_s": round(fps, 1)}
        log(f"{name.replace('_', ' ')} ({W}x{H} -> {wt}x{Ht}): {fps:.1f} frames/s")
    del fr
    return out


def _oracle_sample(args):
    """Whole oracle retarget of the first nf frames of a workload clip (the
    clip regenerated here, so that nothing large crosses processes);
    returns (frames, seconds of the oracle call alone)."""
    workload, index, nf = args
    import numpy as np

    import oracle
    clip, Wt, k = _workload_clip(workload, index)
    clip = np.ascontiguousarray(clip[:nf])
    t0 = time.perf_counter()
    oracle.retarget(clip, Wt, k, mode=1, use_buffer=1, anum=1, aden=5, want_masks=False)
    return clip.shape[0], time.perf_counter() - t0


def _workload_clip(workload, index):
    """Clip `index` of a workload with its target width and seams per
    iteration (as make_workload draws them)."""
    from paper_1903_03180_amd import synth
    if workload == "1080p-batch16":
        return synth.clip_1080p(2000 + index), 1440, 16
    if workload == "1080p":
        return synth.clip_1080p(2), 1440, 16
    if workload == "mix64":
        sp = synth.batch_mix_specs(64)[index]
        return synth.clip_from_spec(sp), sp.Wt, 16
    return synth.clip_4k(3), 2880, 32


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def job_rows(log_rows, jobs):
    """Splits the per-iteration log into the jobs (buffers, in order): a
    job's records continue while its width minus the seams of its previous
    iteration stays above its target."""
    out, j, prev = [[] for _ in jobs], -1, None
    for row in log_rows.tolist():
        _b, Wr, _p, kk = row
        if prev is None or prev[1] - prev[3] <= jobs[j]["Wt"]:
            j += 1
        out[j].append(row)
        prev = row
    return out


def balg_bytes(per_job, jobs):
    """Algorithmic HBM bytes of one step by the paper-literal accounting:
    every input frame read and every output frame written once (plus the
    luma of colour frames), and for every iteration r >= 1 of a buffer each
    of its frames' carved luma re-read for the energy recompute."""
    total = 0
    for rows, jb in zip(per_job, jobs):
        H, W, Wt, C, T = jb["H"], jb["W"], jb["Wt"], jb["C"], jb["T"]
        total += T * (H * W * C + H * Wt * C + (H * W if C == 3 else 0))
        total += T * sum(H * int(r[1]) for r in rows[1:])
    return total


def dp_bytes(per_job, jobs):
    """Algorithmic bytes of the DP over one retarget: per iteration of a
    buffer at width W_r, the 2-byte key of every carved pixel is read once
    and its 1-byte indicator code written once."""
    return sum(3 * jb["H"] * int(r[1]) for rows, jb in zip(per_job, jobs) for r in rows)


def dp_kernel_name(g):
    """rocprofv3 name of the DP kernel of geometry g (ctx.dp_chosen)."""
    kind = "dp_chunk_kernel" if g["chunk_rows"] else "dp_band_kernel"
    return f"{kind}<{g['cols_per_lane']}, {g['halo_rows']}, {g['prefetch_rows']}>"


def measured_dp_traffic(workload, g):
    """HBM bytes per DP (all its dispatches) from the committed FETCH_SIZE / WRITE_SIZE
    runs (scaled by the 1 GiB copy), if they were taken on this workload
    with this DP kernel and the kernel source has not changed since; else
    None."""
    path = os.path.join(ROOT, "profiles", f"dp_traffic_{workload.replace('-', '_')}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    same = dp_source_digest() == rec.get("dp_source_sha256")
    if not same or rec["kernel"] != dp_kernel_name(g) or rec.get("chunk_rows", 0) != g["chunk_rows"] \
            or rec.get("chunk_cols", 0) != g["chunk_cols"]:
        return None
    # a DP of a chunked geometry is one dispatch per chunk of rows
    return (rec["read_bytes_per_dispatch"] + rec["write_bytes_per_dispatch"]) * rec.get("dispatches_per_dp", 1)


def measured_step_traffic(workload, g, variants=None):
    """The committed whole-step counter record of this workload, if it was
    taken with this DP geometry and no kernel or host source has changed
    since; else None."""
    path = os.path.join(ROOT, "profiles", f"step_traffic_{workload.replace('-', '_')}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sources_sha256") != sources_digest() or rec.get("dp_geometry") != g:
        return None
    if variants is not None and rec.get("variants") != variants:
        return None
    return rec


def sources_digest() -> str:
    """SHA-256 over the library's kernel and host sources."""
    import hashlib
    h = hashlib.sha256()
    for name in ("scpl_kernels.hip", "scpl_host.hip", "scpl_internal.h", "scpl_runtime.h"):
        with open(os.path.join(ROOT, "paper_1903_03180_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def dp_source_digest() -> str:
    """SHA-256 of the DP section of the kernel source (key rows, row step,
    code stores, the DP kernels): a traffic record stays valid while that
    text is unchanged."""
    import hashlib
    src = os.path.join(ROOT, "paper_1903_03180_amd", "csrc", "scpl_kernels.hip")
    with open(src) as f:
        text = f.read()
    a = text.index("// ------------------------------------------------------------------- DP")
    b = text.index("// ----------------------------------------------------------- band origins")
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="1080p-batch16", choices=["1080p-batch16", "1080p", "4k", "mix64"])
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--streams", type=int, default=3, help="job groups (streams) of the batched path")
    ap.add_argument("--serve-requests", type=int, default=400, help="requests per arrival rate (0: no serving run)")
    ap.add_argument("--no-table1", action="store_true", help="skip the Proposed-vs-Raw runs on Table 1 shapes")
    ap.add_argument("--mix-leg", type=int, default=1,
                    help="also time the 64 clips of uneven size (batched and plain) after the main workload")
    ap.add_argument("--steps-mix", type=int, default=2, help="timed batched steps of the uneven-mix leg")
    ap.add_argument("--no-height", action="store_true", help="skip the height (horizontal seam) runs")
    ap.add_argument("--cpu-frames", type=int, default=0,
                    help="frames of the oracle's bounded sample (0: 61 for the 1080p workloads, i.e. the first "
                         "buffer and the one-frame buffer of the scene cut; 8 for 4k; 30 for mix64)")
    ap.add_argument("--cpu-procs", type=int, default=16, help="most processes of the all-cores oracle leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dp-geometry", default="", metavar="Q,HB,PF,EX,R,P",
                    help="use this DP geometry instead of autotuning (e.g. under a profiler, whose per-dispatch "
                         "overhead distorts the autotuner's timings)")
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="skip the batch autotuner (job groups, DP geometry and kernel variants timed on whole steps)")
    ap.add_argument("--variants", default="", metavar="UPDATE,REFRESH,BORG,GATHER,FUSE",
                    help="compaction, refresh, band-origin, gather and fused kernel variants to use (with "
                         "--dp-geometry, for profiled runs)")
    ap.add_argument("--memo-periods", default="2,4",
                    help="seam-memorisation periods to time on the same workload (empty: none)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device tensor copy of this many MiB (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import multiprocessing as mp

    import numpy as np

    # the oracle's one-core leg runs in a fresh process beside the GPU legs
    # (spawned before this process touches the GPU)
    cpu_frames = args.cpu_frames or {"4k": 8, "mix64": 30}.get(args.workload, 61)
    cpu_pool = cpu_job = None
    if not args.no_cpu:
        cpu_pool = mp.get_context("spawn").Pool(1)
        cpu_job = cpu_pool.apply_async(_oracle_sample, ((args.workload, 0, cpu_frames),))

    import torch

    from paper_1903_03180_amd import scpl

    t_gen = time.perf_counter()
    work, wname = make_workload(args.workload)
    clips_np = [w[0] for w in work]
    n_frames = sum(c.shape[0] for c in clips_np)
    Hmax = max(c.shape[1] for c in clips_np)
    Wmax = max(c.shape[2] for c in clips_np)
    log(f"workload {wname}; generated {sum(c.nbytes for c in clips_np) / 1e9:.2f} GB in "
        f"{time.perf_counter() - t_gen:.1f} s")
    ctx = scpl.Context(0)
    ctx.batch_streams(args.streams)
    clips = []
    for c, wt, kk in work:
        fr = torch.from_numpy(c).cuda()
        clips.append(dict(frames=fr, target_width=wt, seams_per_iter=kk, alpha_num=1, alpha_den=5,
                          out=torch.empty((c.shape[0], c.shape[1], wt) + c.shape[3:], dtype=torch.uint8,
                                          device="cuda"),
                          buffer_id=torch.empty(c.shape[0], dtype=torch.int32, device="cuda")))
    torch.cuda.synchronize()
    # workloads with committed counter profiles time the configuration the
    # profiles were taken in (the library's defaults)
    profiled = os.path.exists(os.path.join(ROOT, "profiles", f"step_traffic_{args.workload.replace('-', '_')}.json"))
    if args.dp_geometry:
        q, hb, pf, ex, r, p = (int(x) for x in args.dp_geometry.split(","))
        ctx.dp_geometry(q, hb, pf, ex)
        ctx.dp_chunking(r, p)
        dpg = ctx.dp_chosen(Wmax)
        log(f"DP geometry forced: {dpg}")
    elif profiled:
        # the library's default geometry for the batch (the one the counter
        # profiles cover); the DP autotuner runs with the batch autotuner
        # below, on a context of its own
        dpg = ctx.dp_chosen(Wmax)
        log(f"DP geometry (default, profiled): {dpg}")
    else:
        # no counter profiles for this workload: the DP geometry tuned for its
        # number of concurrent jobs (and, for the plain path of a single clip,
        # the nearest tuned job count)
        dpus = ctx.autotune_dp(Hmax, Wmax, n_jobs=min(3 * len(clips), 256))[4]
        dpg = ctx.dp_chosen(Wmax)
        log(f"DP autotune for {min(3 * len(clips), 256)} jobs of {Hmax}x{Wmax}: {dpg}: {dpus:.1f} us per DP")

    # the batch autotuner (whole steps of this workload under each candidate
    # configuration: job groups, DP geometry, kernel variants, the persistent
    # launch) on a context of its own, and its pick timed there.  On this
    # workload its picks differ from the library's defaults by less than the
    # run-to-run noise, so the timed region below runs the defaults: the
    # configuration the committed counter profiles were taken in.
    batch_choice = None
    batch_tuned = None
    if args.variants:
        ctx.kernel_variants(*(int(x) for x in args.variants.split(",")))
    if not args.dp_geometry and not args.no_batch_tune:
        tctx = scpl.Context(0)
        try:
            b0 = time.perf_counter()
            nj_dp = min(3 * len(clips), 256)
            dpus = tctx.autotune_dp(Hmax, Wmax, n_jobs=nj_dp)[4]
            dp_tuned = {"jobs": nj_dp, "geometry": tctx.dp_chosen(Wmax), "us_per_dp": round(dpus, 1)}
            log(f"DP autotune for {nj_dp} jobs of {Hmax}x{Wmax}: {dp_tuned['geometry']}: {dpus:.1f} us per DP")
            batch_choice = tctx.autotune_batch(clips, reps=2)
            log(f"batch autotune ({time.perf_counter() - b0:.1f} s): {batch_choice}")
            tctx.retarget_batch(clips)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                tctx.retarget_batch(clips)
            torch.cuda.synchronize()
            tms = (time.perf_counter() - t0) * 1e3 / args.steps
        finally:
            tctx.close()
        batch_tuned = {"dp_autotune": dp_tuned, "choice": batch_choice, "ms_per_step": round(tms, 3),
                       "fps": round(n_frames / (tms * 1e-3), 2),
                       "timing": "graph-replayed steps in the autotuner's configuration, on a context of its own"}
        log(f"autotuned configuration: {tms:.2f} ms/step, {batch_tuned['fps']:.1f} frames/s")
    # the timed region measures the job-group path (its DP launches carry the
    # roofline); the persistent launch is timed on its own below
    ctx.batch_mode(scpl.SCPL_BATCH_GROUPS)

    def step_batched():
        ctx.retarget_batch(clips)

    for i in range(args.warmup):
        step_batched()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    # timed region: every DP launch bracketed by HIP events on its stream
    # (the roofline's launch time); the other kernels run without events
    ctx.profile(True, kinds=["dp"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dp = ctx.profile_read()["dp"]
    ctx.profile(False)
    log_rows = ctx.last_log()
    nbuf = sum(int(c["buffer_id"].max().item()) + 1 for c in clips)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fps = n_frames * args.steps / (t1 - t0)
    log(f"batched: {ms_per_step:.2f} ms/step, {fps:.1f} frames/s, {nbuf} buffers, "
        f"{len(log_rows)} buffer-iterations")

    # per-kernel breakdown: one more step with every launch bracketed (not
    # part of the timed region; the events slow the step down)
    ctx.profile(True)
    step_batched()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    log("kernel time per step, every launch timed (ms): " +
        ", ".join(f"{kn}={v[0]:.3f}" for kn, v in prof.items() if v[1]))

    # graph-replayed timing of the same batched step (no per-launch events)
    g0 = time.perf_counter()
    for i in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    fps_graph = n_frames * args.steps / (g1 - g0)
    log(f"batched (graph, no event timing): {(g1 - g0) * 1e3 / args.steps:.2f} ms/step, {fps_graph:.1f} frames/s")

    persistent = run_persistent_leg(torch, scpl, ctx, step_batched, n_frames, args.steps, fps_graph, batch_choice)

    # seam memorisation (only buffers b with b mod m == 0 carved): graph-timed
    # steps of the same workload, and how much of the output it changes
    memo = []
    periods = [int(x) for x in args.memo_periods.split(",") if x.strip()]
    if periods:
        full = [c["out"].clone() for c in clips]
        for m in periods:
            for c in clips:
                c["memo_period"] = m
            step_batched()
            torch.cuda.synchronize()
            m0 = time.perf_counter()
            for i in range(args.steps):
                step_batched()
            torch.cuda.synchronize()
            m1 = time.perf_counter()
            diff = sum(int((c["out"] != f).sum().item()) for c, f in zip(clips, full))
            total = sum(f.numel() for f in full)
            nb_carved = sum(len([b for b in range(int(c["buffer_id"].max().item()) + 1) if b % m == 0])
                            for c in clips)
            memo.append({"period": m, "fps_graph": round(n_frames * args.steps / (m1 - m0), 2),
                         "ms_per_step": round((m1 - m0) * 1e3 / args.steps, 3), "buffers_carved": nb_carved,
                         "output_bytes_changed_frac": round(diff / total, 5)})
            log(f"memorisation m={m}: {(m1 - m0) * 1e3 / args.steps:.2f} ms/step, "
                f"{n_frames * args.steps / (m1 - m0):.1f} frames/s, {nb_carved} buffers carved, "
                f"{diff / total:.4f} of output bytes changed")
        for c in clips:
            c["memo_period"] = 0
        del full

    # dominant kernel and its roofline
    ktime = {kn: v[0] for kn, v in prof.items()}
    dom = max(ktime, key=ktime.get)
    dp_ms, dp_n = prof_dp
    dp_launch_ms = dp_ms / max(dp_n, 1)
    jobs = []
    for c, (cnp, wt, kk) in zip(clips, work):
        for T in np.bincount(c["buffer_id"].cpu().numpy()).tolist():
            jobs.append(dict(H=cnp.shape[1], W=cnp.shape[2], Wt=wt, C=cnp.shape[3] if cnp.ndim == 4 else 1, T=T))
    per_job = job_rows(log_rows, jobs)
    dp_bytes_launch = dp_bytes(per_job, jobs) * args.steps / max(dp_n, 1)
    achieved = dp_bytes_launch / (dp_launch_ms * 1e-3) / 1e9
    traffic = measured_dp_traffic(args.workload, dpg)

    # plain path: clips one after another, buffers one after another
    plain_fps = None
    if args.plain_steps > 0:
        if not args.dp_geometry and len(clips) > 1:  # the plain path runs one buffer at a time
            ctx.autotune_dp(Hmax, Wmax, n_jobs=1)
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            for c in clips:
                ctx.retarget(c["frames"], c["target_width"], c["seams_per_iter"], want_masks=False, alpha_num=1,
                             alpha_den=5)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        plain_fps = n_frames * args.plain_steps / (p1 - p0)
        log(f"plain: {(p1 - p0) * 1e3 / args.plain_steps:.2f} ms/step, {plain_fps:.1f} frames/s")

    if args.copy_calibration > 0:
        # kernels of known traffic for scaling the hardware byte counters: a
        # copy (n read, n written); a sum of the int32 view into int64, which
        # torch runs as a conversion (n read, 2n written) and a reduction (2n
        # read); a fill (n written)
        nb = args.copy_calibration << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        total = int(a.view(torch.int32).sum(dtype=torch.int64).item())
        b.fill_(2)
        torch.cuda.synchronize()
        log(f"calibration: copy of {args.copy_calibration} MiB, sum of {args.copy_calibration} MiB "
            f"(= {total}), fill of {args.copy_calibration} MiB")
        del a, b

    # paper-literal algorithmic bytes per step
    balg = balg_bytes(per_job, jobs)
    # VALU busy per kernel, from the committed counter run (same sources)
    valu_busy = None
    vpath = os.path.join(ROOT, "profiles", f"valu_busy_{args.workload.replace('-', '_')}.json")
    if os.path.exists(vpath):
        with open(vpath) as f:
            vrec = json.load(f)
        if vrec.get("sources_sha256") == sources_digest():
            valu_busy = {"source": "rocprofv3 VALUBusy per dispatch (each dispatch alone), profiles/" +
                                   vrec["summary"], "per_kernel": vrec["valu_busy"]}
    # HBM bytes a step actually moves, from the committed counter runs
    step_hbm = None
    variants = None
    if args.variants:
        variants = [int(x) for x in args.variants.split(",")]
    step_rec = measured_step_traffic(args.workload, dpg, variants or [0, 0, 0, 4, 0])
    if step_rec is not None:
        gbs = step_rec["bytes_per_step"] / (ms_per_step * 1e-3) / 1e9
        step_hbm = {"source": "rocprofv3 FETCH_SIZE + WRITE_SIZE over every dispatch of a step (calibrated), "
                              "profiles/" + step_rec["summary"],
                    "bytes_per_step": step_rec["bytes_per_step"], "GBps": round(gbs, 1),
                    "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}

    table1 = None if args.no_table1 else run_table1(np, torch, scpl, ctx)
    height = None if args.no_height else run_height(torch, ctx, clips_np[0], work[0][1], work[0][2], 2)

    serving = None
    n_clips = n_clips_all = len(clips)
    shape = {"height": Hmax, "width": Wmax, "target_width": work[0][1], "seams_per_iter": work[0][2]} \
        if len({(c.shape[1:], w, kk) for c, w, kk in work}) == 1 else {"uneven": True}
    mix = None
    if args.serve_requests > 0 or (args.mix_leg and args.workload != "mix64"):
        del clips, clips_np, work
        torch.cuda.empty_cache()
    if args.mix_leg and args.workload != "mix64":
        mix = run_mix(np, torch, ctx, args.steps_mix)
    if args.serve_requests > 0:
        serving = run_serving(np, torch, scpl, n_req=args.serve_requests)

    # the oracle: its one-core leg has run beside the GPU legs; then every
    # usable core (up to --cpu-procs), one process per clip on the same
    # sample of each clip
    cpu = cpu_all = None
    if cpu_job is not None:
        nf, secs = cpu_job.get()
        cpu_pool.close()
        cpu_pool.join()
        where = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": usable_cores()}
        sample = (f"the first {nf} frames of the first clip of the workload, retargeted whole by the oracle "
                  f"(segmentation and every iteration of each of the sample's buffers; for the 1080p clips the "
                  f"workload's first buffer, 60 frames, and the one-frame buffer of the scene cut), "
                  f"{secs:.1f} s on one core")
        cpu = {"value": round(nf / secs, 4), "unit": "frames/s", "cores": 1, "kind": "oracle", "sample": sample,
               **where}
        log(f"oracle: {nf} frames in {secs:.1f} s on one core ({where['cpu_model']}, nproc {where['nproc']})")
        procs = max(1, min(args.cpu_procs, usable_cores(), n_clips_all))
        with mp.get_context("spawn").Pool(procs) as pool:
            c0 = time.perf_counter()
            res = pool.map(_oracle_sample, [(args.workload, i, cpu_frames) for i in range(procs)])
            c1 = time.perf_counter()
        done = sum(r[0] for r in res)
        slowest = max(r[1] for r in res)
        cpu_all = {"value": round(done / slowest, 4), "unit": "frames/s", "cores": procs, "kind": "oracle",
                   "sample": f"the same sample of each of the first {procs} clips, one process per clip, all "
                             f"started together: {done} frames; the slowest process's oracle call took "
                             f"{slowest:.1f} s ({c1 - c0:.1f} s with start-up and clip generation)",
                   **where}
        log(f"oracle on {procs} cores: {done} frames, slowest oracle call {slowest:.1f} s")

    line = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/int32",
        "data": "synthetic",
        "config": {"workload": wname, "path": "batched: all buffers of all clips per launch, HIP-graph iterations",
                   "clips": n_clips, "frames": n_frames, **shape, "buffers": nbuf,
                   "buffer_iterations": int(len(log_rows)),
                   "dp_geometry": dpg,
                   "streams": args.streams,
                   "variants": [int(x) for x in args.variants.split(",")] if args.variants else "defaults",
                   "batch_tuning": batch_tuned},
        "value_graph_no_events": round(fps_graph, 2),
        "plain_fps": None if plain_fps is None else round(plain_fps, 2),
        "batched_over_plain": None if plain_fps is None else round(fps / plain_fps, 3),
        "kernel_ms_per_step": {kn: round(v[0], 4) for kn, v in prof.items() if v[1]},
        "dominant_kernel": dom,
        "roofline": {"kernel": "dp", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(dp_bytes_launch), "launch_ms": round(dp_launch_ms, 4)},
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "hbm_measured": step_hbm,
        "valu_busy": valu_busy,
        "paper_literal_bytes": {
            "accounting": "algorithmic, not measured: input read, output written, colour luma written, and the "
                          "carved luma re-read by every frame of a buffer at every iteration >= 1 (the full "
                          "energy recompute the partial refresh never performs)",
            "bytes_per_step": int(balg), "GBps": round(balg / (ms_per_step * 1e-3) / 1e9, 1),
            "frac_of_peak": round(balg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "persistent": persistent,
        "mix64": mix,
        "serving": serving,
        "raw_vs_proposed": table1,
        "seam_memorisation": memo,
        "horizontal_seams": height,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
