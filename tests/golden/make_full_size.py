"""Writes full_size_sha256.json: SHA-256 digests of the CPU oracle's whole
retarget of the full-size workloads, every iteration of every buffer
included.

Only the oracle (oracle/) computes anything here; the clips come from the
seeded generator (paper_1903_03180_amd/synth.py, which holds no retargeting
arithmetic).  For each workload the file records the recipe, the buffer
lengths, the number of logged iterations, and the digests of the output
frames, the masks, the buffer ids and the per-iteration log (buffer, W_r,
P_eff, k_iter), each taken over the array's bytes in C order with its dtype
as stored by oracle.retarget (out uint8, masks uint16, buffer ids and log
int32).

Workloads (Secs. 3.1-3.3 at the sizes of the measured configurations):
  clip1080p_s2        1080p RGB clip, 120 frames, cut at 60, 1920 -> 1440, k 16, alpha 1/5
  clip1080p_s2000..   the 16 clips of the 1080p batch (same generator), same targets
  clip4k_s3_a<n>_<d>  4K luma clip, 60 frames, pan, 3840 -> 2880, k 32, alpha n/d in {3/20, 1/5, 1/4}
  mix_<seed>          the first 16 clips of the uneven mix, luma, W -> floor(3W/4), k 16, alpha 1/5

Usage: python tests/golden/make_full_size.py [-j JOBS] [names...]
Each workload runs in its own process (the oracle is single-threaded);
existing entries are kept unless named again.  The whole set takes about
an hour of CPU time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full_size_sha256.json")

HEADLINE_SEEDS = list(range(2000, 2016))
ALPHAS_4K = [(3, 20), (1, 5), (1, 4)]
N_MIX = 16


def workloads() -> dict:
    w = {"clip1080p_s2": dict(kind="1080p", seed=2, Wt=1440, k=16, anum=1, aden=5)}
    for s in HEADLINE_SEEDS:
        w[f"clip1080p_s{s}"] = dict(kind="1080p", seed=s, Wt=1440, k=16, anum=1, aden=5)
    for a, d in ALPHAS_4K:
        w[f"clip4k_s3_a{a}_{d}"] = dict(kind="4k", seed=3, Wt=2880, k=32, anum=a, aden=d)
    from paper_1903_03180_amd import synth
    for s in synth.batch_mix_specs(64)[:N_MIX]:
        w[f"mix_{s.seed}"] = dict(kind="mix", seed=s.seed, N=s.N, H=s.H, W=s.W, Wt=s.Wt, k=16, anum=1, aden=5)
    return w


def frames_of(rec):
    from paper_1903_03180_amd import synth
    if rec["kind"] == "1080p":
        return synth.clip_1080p(rec["seed"])
    if rec["kind"] == "4k":
        return synth.clip_4k(rec["seed"])
    spec = synth.ClipSpec(rec["seed"], rec["N"], rec["H"], rec["W"], rec["Wt"])
    return synth.clip_from_spec(spec)


def sha(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run_one(item):
    name, rec = item
    import numpy as np
    import oracle
    fr = frames_of(rec)
    t0 = time.time()
    res = oracle.retarget(fr, rec["Wt"], rec["k"], anum=rec["anum"], aden=rec["aden"])
    dt = time.time() - t0
    entry = dict(recipe=rec, shape=list(fr.shape),
                 buffers=np.bincount(res["buffer_id"]).tolist(),
                 iterations=int(len(res["log"])),
                 sha256=dict(out=sha(res["out"]), masks=sha(res["masks"]),
                             buffer_id=sha(res["buffer_id"]), log=sha(res["log"])),
                 oracle_seconds=round(dt, 1))
    print(f"{name}: {dt:.1f} s, buffers {entry['buffers']}, {entry['iterations']} iterations", flush=True)
    return name, entry


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    w = workloads()
    names = a.names or list(w)
    for n in names:
        if n not in w:
            raise SystemExit(f"unknown workload {n}")
    have = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            have = json.load(f)["workloads"]
    # longest first, so the pool's tail is short
    order = sorted(names, key=lambda n: -{"4k": 4, "1080p": 2}.get(w[n]["kind"], 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(a.jobs, maxtasksperchild=1) as pool:
        for name, entry in pool.imap_unordered(run_one, [(n, w[n]) for n in order]):
            have[name] = entry
            doc = {"about": "SHA-256 of the CPU oracle's whole retarget of full-size workloads; "
                            "written by tests/golden/make_full_size.py, which calls only oracle/ "
                            "(inputs from the seeded generator)",
                   "workloads": dict(sorted(have.items()))}
            tmp = OUT + ".tmp"
            with open(tmp, "w") as f:
                json.dump(doc, f, indent=1, sort_keys=True)
                f.write("\n")
            os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
