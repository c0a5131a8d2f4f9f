"""Benchmark: SCPL video retargeting of a 1080p clip on one MI355X.

A step is one whole retarget of the workload clip (luma, buffer
segmentation, every SCPL iteration of every buffer, output gather) with the
frames already resident in HBM.  The reported value is frames per second of
the batched path (all buffers of the clip advance together, one launch per
stage per iteration); the plain path (one buffer after another) is timed
beside it.  The oracle (plain C, one core) is timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1080p|4k]
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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def energy_bytes(log_rows, bid, H, mode):
    """Algorithmic bytes of the energy kernel over one retarget: per
    iteration of a buffer of T frames at width W_r, every carved pixel of
    every frame (plus the predecessor of the first frame in motion mode) is
    read once (1 B), the column map is read once (2 B per carved pixel) and
    the uniform energy written once (2 B per carved pixel)."""
    import numpy as np
    starts = {}
    for t in range(len(bid)):
        b = int(bid[t])
        if b not in starts:
            starts[b] = [t, 0]
        starts[b][1] += 1
    total = 0
    for b, Wr, _peff, _kk in log_rows.tolist():
        t0, T = starts[b]
        frames = T + (1 if (mode == 1 and t0 > 0) else 0)
        total += frames * H * Wr + 4 * H * Wr
    return total


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="1080p", choices=["1080p", "4k"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-frames", type=int, default=4, help="frames of the oracle's bounded sample")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1903_03180_amd import scpl, synth

    if args.workload == "1080p":
        frames_np = synth.clip_1080p(2)
        Wt, k, anum, aden = 1440, 16, 1, 5
        wname = "1080p RGB clip: 120 frames 1920x1080 -> 1440 wide, k=16 seams/iteration, alpha=1/5, motion energy"
    else:
        frames_np = synth.clip_4k(3)
        Wt, k, anum, aden = 2880, 32, 1, 5
        wname = "4K luma clip: 60 frames 3840x2160 -> 2880 wide, k=32 seams/iteration, alpha=1/5, motion energy"
    N, H, W = frames_np.shape[:3]
    log(f"workload {wname}; generated {frames_np.nbytes / 1e6:.0f} MB")
    frames = torch.from_numpy(frames_np).cuda()
    out = torch.empty((N, H, Wt) + frames_np.shape[3:], dtype=torch.uint8, device="cuda")
    bid = torch.empty(N, dtype=torch.int32, device="cuda")
    ctx = scpl.Context(0)
    clip = dict(frames=frames, target_width=Wt, seams_per_iter=k, alpha_num=anum, alpha_den=aden, out=out,
                buffer_id=bid)

    def step_batched():
        ctx.retarget_batch([clip])

    for i in range(args.warmup):
        step_batched()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    log_rows = ctx.last_log()
    bid_np = bid.cpu().numpy()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    fps = N * args.steps / (t1 - t0)
    log(f"batched: {ms_per_step:.2f} ms/step, {fps:.1f} frames/s, {int(bid_np.max()) + 1} buffers, "
        f"{len(log_rows)} buffer-iterations")

    # dominant kernel and its roofline
    ktime = {kname: v[0] for kname, v in prof.items()}
    dom = max(ktime, key=ktime.get)
    e_ms, e_n = prof["energy"]
    e_bytes_step = energy_bytes(log_rows, bid_np, H, 1)
    e_launch_ms = e_ms / max(e_n, 1)
    e_bytes_launch = e_bytes_step * args.steps / max(e_n, 1)
    achieved = e_bytes_launch / (e_launch_ms * 1e-3) / 1e9
    log("kernel time per step (ms): " + ", ".join(f"{kn}={v[0] / args.steps:.3f}" for kn, v in prof.items() if v[1]))

    # plain path
    plain_fps = None
    if args.plain_steps > 0:
        ctx.retarget(frames, Wt, k, want_masks=False, alpha_num=anum, alpha_den=aden)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            ctx.retarget(frames, Wt, k, want_masks=False, alpha_num=anum, alpha_den=aden)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        plain_fps = N * args.plain_steps / (p1 - p0)
        log(f"plain: {(p1 - p0) * 1e3 / args.plain_steps:.2f} ms/step, {plain_fps:.1f} frames/s")

    cpu = None
    if not args.no_cpu:
        import oracle
        nf = min(args.cpu_frames, N)
        c0 = time.perf_counter()
        oracle.retarget(frames_np[:nf], Wt, k, mode=1, use_buffer=1, anum=anum, aden=aden, want_masks=False)
        c1 = time.perf_counter()
        cpu = {"value": round(nf / (c1 - c0), 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"first {nf} frames of the same clip, whole retarget (segmentation + every iteration), "
                         f"{c1 - c0:.1f} s on one core"}
        log(f"oracle: {nf} frames in {c1 - c0:.1f} s")

    line = {
        "metric": "1080p frames/s (batched vs plain, bit-exact); HBM GB/s; p50/p99 latency",
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
        "config": {"workload": wname, "path": "batched (all buffers per launch)", "frames": N, "height": H,
                   "width": W, "target_width": Wt, "seams_per_iter": k,
                   "buffers": int(bid_np.max()) + 1, "buffer_iterations": int(len(log_rows))},
        "plain_fps": None if plain_fps is None else round(plain_fps, 2),
        "batched_over_plain": None if plain_fps is None else round(fps / plain_fps, 3),
        "kernel_ms_per_step": {kn: round(v[0] / args.steps, 4) for kn, v in prof.items() if v[1]},
        "dominant_kernel": dom,
        "roofline": {"kernel": "energy", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(e_bytes_launch), "launch_ms": round(e_launch_ms, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
