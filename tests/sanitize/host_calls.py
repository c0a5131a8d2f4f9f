"""Host-side entry points of libscpl.so that need no GPU, called on many
argument sets: parameter validation, workspace and admission arithmetic,
status strings, and every entry point with a null context or null
pointers (each must return an error status without touching memory).
Run under AddressSanitizer / UndefinedBehaviorSanitizer by
tests/test_sanitizers.py with the library path as argv[1]."""
import ctypes as C
import itertools
import sys

L = C.CDLL(sys.argv[1])


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "n_frames", "height", "width", "channels", "target_width", "seams_per_iter", "energy_mode",
        "use_buffer", "alpha_num", "alpha_den", "max_buffer", "target_height", "memo_period")]


n = 0
b = C.c_uint64()
for N, H, W, Ch, Wt, k, mode, ub, an, ad, mb, th, memo in itertools.product(
        [0, 1, 7, 16384, 16385], [0, 1, 9, 1080, 32767], [0, 1, 17, 1920, 32767], [1, 2, 3], [0, 1, 8, 1440, 40000],
        [0, 1, 16, 40000], [1, 2], [1], [1, 2000], [5], [0, 3], [0, 5], [0, 3]):
    p = Params(N, H, W, Ch, Wt, k, mode, ub, an, ad, mb, th, memo)
    L.scpl_workspace_size(C.byref(p), C.byref(b))
    L.scpl_server_footprint(C.byref(p), C.byref(b))
    n += 1
L.scpl_status_str.restype = C.c_char_p
for s in range(-3, 10):
    assert L.scpl_status_str(s)
p = Params(4, 8, 16, 1, 12, 2, 1, 1, 1, 5, 0, 0, 0)
nul = None
i32, i64, dbl = C.c_int32(), C.c_int64(), C.c_double()
calls = [
    lambda: L.scpl_create(0, nul),
    lambda: L.scpl_workspace_size(nul, C.byref(b)),
    lambda: L.scpl_workspace_size(C.byref(p), nul),
    lambda: L.scpl_retarget(nul, C.byref(p), nul, nul, nul, nul, nul, nul, C.c_uint64(0), nul),
    lambda: L.scpl_retarget_noalloc(nul, C.byref(p), nul, nul, nul, nul, nul, nul),
    lambda: L.scpl_retarget_batch(nul, nul, 0, nul),
    lambda: L.scpl_kernel_variants(nul, 0, 0, 0, 0, 0),
    lambda: L.scpl_batch_mode(nul, 1),
    lambda: L.scpl_persist_stats(nul, None, None),
    lambda: L.scpl_device_xcds(nul, None),
    lambda: L.scpl_persist_workgroups(nul, 0),
    lambda: L.scpl_autotune_batch(nul, nul, 1, 1, nul, nul, nul),
    lambda: L.scpl_batch_streams(nul, 1),
    lambda: L.scpl_last_log(nul, nul, C.c_int64(0), C.byref(i64)),
    lambda: L.scpl_profile_enable(nul, 1),
    lambda: L.scpl_profile_kinds(nul, 1),
    lambda: L.scpl_profile_read(nul, 0, C.byref(dbl), C.byref(i64)),
    lambda: L.scpl_dp_geometry(nul, 4, 16, 8, 1),
    lambda: L.scpl_dp_chunking(nul, 256, 384),
    lambda: L.scpl_dp_chosen(nul, 100, nul),
    lambda: L.scpl_autotune_dp(nul, 8, 8, 1, nul, nul, nul, nul, nul),
    lambda: L.scpl_luma(nul, nul, C.c_int64(4), nul, nul),
    lambda: L.scpl_energy(nul, 4, 4, 0, nul, nul, nul, nul),
    lambda: L.scpl_dp(nul, 4, 4, nul, nul, nul, nul, nul),
    lambda: L.scpl_select(nul, 4, nul, nul, 1, 1, nul, nul, nul, nul),
    lambda: L.scpl_backtrack(nul, 4, 4, nul, nul, 1, nul, nul),
    lambda: L.scpl_asde(nul, 2, 4, 4, 1, nul, nul, 1, 5, nul, nul, nul),
    lambda: L.scpl_compact(nul, 4, 4, 1, nul, nul, 1, nul, nul),
    lambda: L.scpl_segment(nul, C.byref(p), nul, nul, nul, nul, nul),
    lambda: L.scpl_server_create(0, nul, nul),
    lambda: L.scpl_server_submit(nul, nul, nul),
    lambda: L.scpl_server_poll(nul, C.c_int64(1), C.byref(i32), nul),
    lambda: L.scpl_server_wait(nul, C.c_int64(1), nul),
    lambda: L.scpl_server_ticket_times(nul, C.c_int64(1), nul, nul),
    lambda: L.scpl_server_release(nul, C.c_int64(1)),
    lambda: L.scpl_server_footprint(nul, C.byref(b)),
]
for f in calls:
    assert f() != 0
L.scpl_destroy(nul)
L.scpl_server_destroy(nul)
print(f"host calls: {n} parameter sets, {len(calls)} null-argument calls: ok")
