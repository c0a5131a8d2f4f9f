"""CPU-side checks of the HIP library: it loads, exports every entry point
declared in include/scpl.h, and validates arguments on the host (no device
work is started by any call here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "scpl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scpl_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1903_03180_amd import scpl
    return scpl


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 13
    raw = C.CDLL(lib.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), s
    assert sorted(lib.EXPORTS) == syms


def test_status_strings(lib):
    for st in range(7):
        assert lib.scpl_status_str(st)
    assert lib.scpl_status_str(0) == b"ok"


def base(**kw):
    from paper_1903_03180_amd.scpl import Params
    p = dict(n_frames=120, height=1080, width=1920, channels=3, target_width=1440, seams_per_iter=16)
    p.update(kw)
    return Params(**p).c()


def wsize(lib, p):
    out = C.c_uint64(0)
    return lib.scpl_workspace_size(C.byref(p), C.byref(out)), out.value


@pytest.mark.parametrize("kw", [
    dict(n_frames=0), dict(n_frames=16385), dict(height=0), dict(width=0), dict(width=32768),
    dict(height=32768), dict(height=30000, width=30000), dict(channels=2), dict(target_width=0),
    dict(target_width=1921), dict(seams_per_iter=0), dict(energy_mode=2), dict(use_buffer=2),
    dict(alpha_num=-1), dict(alpha_den=0), dict(alpha_num=1025), dict(alpha_den=1025), dict(max_buffer=-1),
    dict(target_height=-1), dict(target_height=1081), dict(memo_period=-1), dict(memo_period=16385),
])
def test_invalid_params_rejected(lib, kw):
    st, _ = wsize(lib, base(**kw))
    assert st == lib.SCPL_ERR_INVALID_ARG


def test_workspace_size_scales(lib):
    st, a = wsize(lib, base())
    assert st == lib.SCPL_OK
    st, b = wsize(lib, base(channels=1))
    assert st == lib.SCPL_OK
    # every clip is held as tiled luma (16 x 8 tiles), whatever its channels
    assert a == b >= 120 * 1080 * 1920
    st, c = wsize(lib, base(height=2160, width=3840, target_width=2880, channels=1, n_frames=60))
    assert c > b
    # a height pass adds its transposed frames
    st, d = wsize(lib, base(target_height=720))
    assert st == lib.SCPL_OK and d > a


def test_workspace_size_covers_the_clip_areas(lib):
    """The plain path holds the clip's luma twice (16 x 8 tiles for the
    stencils, pixel-major 16-frame pieces for the refresh: N + 1 entries per
    pixel rounded up to 16), the segmentation's moments (S1 in 32 bits, S2 in
    64), the first key rows of up to four buffers that the segmentation
    leaves, and one job per buffer at a time."""
    N, H, W = 120, 1080, 1920
    st, a = wsize(lib, base())
    tiled = N * ((H + 15) // 16) * ((W + 7) // 8) * 128
    seq = H * W * ((N + 1 + 15) // 16 * 16)
    seg = H * W * (4 + 8) + 4 * H * W * 2
    job = H * W * (2 + 2 + 1 + 2)  # column map, key rows, indicator codes, mask
    assert a >= tiled + seq + seg + job
    assert a < tiled + seq + seg + 3 * job


def test_null_context_and_pointers_rejected(lib):
    p = base()
    nb = C.c_int32(0)
    assert lib.scpl_retarget(None, C.byref(p), 1, 1, None, None, C.byref(nb), None, 0, None) == \
        lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_retarget_batch(None, None, 0, None) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_create(0, None) == lib.SCPL_ERR_INVALID_ARG
    n = C.c_int64(0)
    assert lib.scpl_last_log(None, None, 0, C.byref(n)) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_profile_kinds(None, 1) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_dp_chunking(None, 256, 384) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_batch_mode(None, lib.SCPL_BATCH_PERSISTENT) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_persist_stats(None, None, None) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_device_xcds(None, None) == lib.SCPL_ERR_INVALID_ARG
    assert lib.scpl_persist_workgroups(None, 0) == lib.SCPL_ERR_INVALID_ARG


def test_target_width_rule_for_batch_mix():
    from paper_1903_03180_amd import synth
    specs = synth.batch_mix_specs(64)
    assert len(specs) == 64
    for s in specs:
        assert 480 <= s.W <= 2560 and 360 <= s.H <= 1440 and s.H % 2 == 0 and 30 <= s.N <= 240
        assert s.Wt == (3 * s.W) // 4
