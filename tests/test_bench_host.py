"""Host-side pieces of the benchmark: the one-GPU refusal, the split of the
iteration log into buffers, the algorithmic byte counts behind `roofline`
and `paper_literal_bytes`, the rules that pair a committed counter record
with the DP (or the step) it was taken on, and the oracle-sample helpers.
Hand-computed values; no GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


JOBS = [dict(H=4, W=10, Wt=6, C=3, T=2), dict(H=4, W=10, Wt=7, C=1, T=5)]
# job 0: widths 10 -> 8 -> 6 (k 2, 2); job 1: 10 -> 9 -> 8 -> 7 (k 1, 1, 1)
LOG = np.array([[0, 10, 5, 2], [0, 8, 3, 2], [1, 10, 4, 1], [1, 9, 4, 1], [1, 8, 2, 1]], dtype=np.int32)


def test_log_split_into_buffers():
    per = bench.job_rows(LOG, JOBS)
    assert [len(r) for r in per] == [2, 3]
    assert [r[1] for r in per[1]] == [10, 9, 8]


def test_dp_bytes_are_three_per_carved_pixel():
    per = bench.job_rows(LOG, JOBS)
    # 3 B x H x W_r over every iteration: job 0 (10 + 8), job 1 (10 + 9 + 8), H = 4
    assert bench.dp_bytes(per, JOBS) == 3 * 4 * (10 + 8) + 3 * 4 * (10 + 9 + 8)


def test_paper_literal_bytes():
    per = bench.job_rows(LOG, JOBS)
    # job 0 (RGB): T (H W C + H Wt C + H W) + T H W_1 ; job 1 (luma): T (H W + H Wt) + T H (W_1 + W_2)
    j0 = 2 * (4 * 10 * 3 + 4 * 6 * 3 + 4 * 10) + 2 * 4 * 8
    j1 = 5 * (4 * 10 + 4 * 7) + 5 * 4 * (9 + 8)
    assert bench.balg_bytes(per, JOBS) == j0 + j1


def test_dp_kernel_names():
    single = dict(cols_per_lane=8, halo_rows=16, prefetch_rows=8, exclusive_cu=1, chunk_rows=0, chunk_cols=0)
    chunked = dict(cols_per_lane=4, halo_rows=16, prefetch_rows=8, exclusive_cu=1, chunk_rows=256, chunk_cols=384)
    assert bench.dp_kernel_name(single) == "dp_band_kernel<8, 16, 8>"
    assert bench.dp_kernel_name(chunked) == "dp_chunk_kernel<4, 16, 8>"


def test_counter_record_matches_only_its_dp():
    path = os.path.join(ROOT, "profiles", "dp_traffic_1080p_batch16.json")
    with open(path) as f:
        rec = json.load(f)
    name = rec["kernel"]
    q, hb, pf = (int(x) for x in name[name.index("<") + 1:-1].split(","))
    g = dict(cols_per_lane=q, halo_rows=hb, prefetch_rows=pf, exclusive_cu=1, chunk_rows=rec.get("chunk_rows", 0),
             chunk_cols=rec.get("chunk_cols", 0))
    want = (rec["read_bytes_per_dispatch"] + rec["write_bytes_per_dispatch"]) * rec.get("dispatches_per_dp", 1)
    if rec["dp_source_sha256"] == bench.dp_source_digest():
        assert bench.measured_dp_traffic("1080p-batch16", g) == want
    else:
        pytest.skip("the DP source changed since the counters were taken")
    other = dict(g, chunk_cols=g["chunk_cols"] + 4)
    assert bench.measured_dp_traffic("1080p-batch16", other) is None
    assert bench.measured_dp_traffic("4k", g) is None


def test_step_record_needs_same_sources_and_geometry(tmp_path, monkeypatch):
    g = dict(cols_per_lane=4, halo_rows=16, prefetch_rows=8, exclusive_cu=1, chunk_rows=256, chunk_cols=384)
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = dict(bytes_per_step=123, dp_geometry=g, sources_sha256=bench.sources_digest(), summary="x.md")
    (prof / "step_traffic_1080p_batch16.json").write_text(json.dumps(rec))
    csrc = tmp_path / "paper_1903_03180_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("scpl_kernels.hip", "scpl_host.hip", "scpl_internal.h", "scpl_runtime.h"):
        (csrc / name).write_bytes(open(os.path.join(ROOT, "paper_1903_03180_amd", "csrc", name), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_step_traffic("1080p-batch16", g)["bytes_per_step"] == 123
    assert bench.measured_step_traffic("1080p-batch16", dict(g, chunk_rows=128)) is None
    assert bench.measured_step_traffic("4k", g) is None
    (csrc / "scpl_host.hip").write_text("changed")
    assert bench.measured_step_traffic("1080p-batch16", g) is None


def test_workload_clip_matches_make_workload():
    from paper_1903_03180_amd import synth
    spec = synth.batch_mix_specs(64)[3]
    clip, wt, k = bench._workload_clip("mix64", 3)
    assert clip.shape[:3] == (spec.N, spec.H, spec.W) and wt == spec.Wt and k == 16


def test_oracle_sample_times_the_oracle():
    n, secs = bench._oracle_sample(("mix64", 0, 2))
    assert n == 2 and secs > 0
    assert bench.usable_cores() >= 1 and isinstance(bench.cpu_model(), str)
